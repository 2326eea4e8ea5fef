// batch_api.cpp -- the batch object of the C ABI (include/gs.h): descriptors and
// task lists in device memory, schedule resolution (fixed or autotuned), and
// replay of the launch sequence through a hipGraph.
//
// All work of a batch runs on a stream the batch owns, ordered after the
// caller's stream by an event and waited for by the caller's stream in turn, so
// the launch sequence can be captured whatever the caller's stream is.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "api_internal.hpp"
#include "autotune.hpp"

using namespace gsapi;

struct gs_batch_s {
    std::vector<gs_plan> plans;
    int device = 0;
    hipStream_t user = nullptr, own = nullptr;
    gs_batch_options req{};
    TuneEntry cfg;
    bool resolved = false, autotuned = false, kernels_ok = true;
    int candidates = 0;
    double tuned_ms = 0.0, points = 0.0;
    int resident = 0;
    // device memory
    void* d_probs = nullptr;
    size_t probs_bytes = 0;
    int* d_tasks = nullptr;
    size_t tasks_cap = 0;                 // ints
    unsigned* d_ctr = nullptr;
    int nctr = 0;
    unsigned char* h_stage = nullptr;     // pinned staging of the descriptors
    unsigned* h_flag = nullptr;           // pinned copy of the error flag, refreshed after each queue launch
    std::vector<unsigned char> probs_dev; // descriptors now in device memory
    int ntasks = 0, pass_off[6] = {}, pass_cnt[6] = {};
    std::vector<int> runs;                // (pass, n, first task, count) of the sized schedule
    int tasks_mult = -1, tasks_lf = -1, tasks_queue = -1;
    gsk::BatchQueueSpec queues;           // the queue schedule's per-die queues
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_staged = nullptr;
    bool staged_pending = false;
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> graph_sig;   // what the captured launches baked in
    // the concurrent schedules: side streams forked from `own` and joined back into it
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_done;
    hipEvent_t ev_fork = nullptr;
};

namespace {

// Side streams of the concurrent schedules (the device's default number of hardware queues).
constexpr int kSideStreams = 4;

// Schedules that run each plan's own launches (no batched kernels, no task list).
bool own_launches(int schedule) { return schedule == GS_SCHED_SEQUENTIAL || schedule == GS_SCHED_STREAMS; }

// Polls of a dependency wait before it gives up (about 2 us each: seconds in all,
// orders of magnitude beyond the longest task).
constexpr unsigned kSpinLimit = 1u << 22;
// Default block-fulls of tiles per task of the queue schedule.
constexpr int kQueueTilesPerTask = 8;

std::mutex g_batch_mu;
std::unordered_set<gs_batch_s*> g_batches;

bool batch_live(gs_batch b) {
    std::lock_guard<std::mutex> g(g_batch_mu);
    return b && g_batches.count(b);
}

void release(gs_batch_s* b) {
    DeviceScope ds(b->device);
    if (b->own) (void)hipStreamSynchronize(b->own);
    for (hipStream_t st : b->side) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : b->side_done) (void)hipEventDestroy(ev);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->d_tasks) (void)hipFree(b->d_tasks);
    if (b->d_ctr) (void)hipFree(b->d_ctr);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->h_flag) (void)hipHostFree(b->h_flag);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->ev_staged) (void)hipEventDestroy(b->ev_staged);
    if (b->own) (void)hipStreamDestroy(b->own);
    delete b;
}

gs_status members(gs_batch_s* b, const double* const* rho, double* const* u, std::vector<gsk::BatchMember>& m) {
    m.resize(b->plans.size());
    for (size_t i = 0; i < b->plans.size(); ++i) {
        gsk::EvalArgs a;
        const gs_status st = make_args(b->plans[i], rho[i], u[i], a);
        if (st != GS_OK) return st;
        gsk::BatchMember& x = m[i];
        x.d = a.d;
        x.n = a.n;
        x.dipolar = a.dipolar;
        x.rho = a.rho;
        x.u = a.u;
        x.X1 = a.X1;
        x.X2 = a.X2;
        x.spec = a.spec;
        x.tw = a.tw;
        for (int i = 0; i < 3; ++i) x.dxi[i] = a.dxi[i];
        for (int k = 0; k < 3; ++k) {
            x.cdiag[k] = a.cdiag[k];
            x.ccross[k] = a.ccross[k];
        }
        x.nm_over_M = a.nm_over_M;
    }
    return GS_OK;
}

// Queues of the queue schedule: one per die the device's blocks run on (problems
// pinned to a die), or a single shared queue if the dies cannot be identified.
void plan_queues(gs_batch_s* b) {
    int ids[32];
    const int c = gsk::batch_xcc_ids(ids, 32);
    gsk::BatchQueueSpec& q = b->queues;
    bool ok = c >= 1 && c <= 16;
    for (int i = 0; i < c && ok; ++i) ok = ids[i] >= 0 && ids[i] < 16;
    for (int i = 0; i < 16; ++i) q.qmap[i] = ok ? -1 : 0;
    if (ok) {
        q.nq = c;
        q.local = 1;
        for (int i = 0; i < c; ++i) q.qmap[ids[i]] = i;
    } else {
        q.nq = 1;
        q.local = 0;
    }
}

// The task list of (schedule, mult, largest_first) in device memory (synchronous: rare).
gs_status upload_tasks(gs_batch_s* b, const std::vector<gsk::BatchMember>& m, int mult, int lf, int schedule) {
    const int queue = schedule == GS_SCHED_QUEUE ? 1 : 0;
    if (b->tasks_mult == mult && b->tasks_lf == lf && b->tasks_queue == queue) return GS_OK;
    std::vector<int> t;
    if (queue) {
        plan_queues(b);
        gsk::batch_queue_tasks(m, mult, b->queues.nq, t, b->queues.qoff);
        for (int p = 0; p < 6; ++p) b->pass_off[p] = b->pass_cnt[p] = 0;
        for (size_t k = 0; k < t.size() / gsk::BATCH_TASK_INTS; ++k)      // field 1 of a task: its pass
            b->pass_cnt[t[k * gsk::BATCH_TASK_INTS + 1]]++;
        b->runs.clear();
    } else {
        gsk::batch_tasks(m, mult, lf != 0, t, b->pass_off, b->pass_cnt);
        gsk::batch_size_runs(m, t, b->runs);
    }
    hipError_t e = hipStreamSynchronize(b->own);
    if (e != hipSuccess) return hip_fail(e, "batch stream");
    if (t.size() > b->tasks_cap) {
        if (b->d_tasks) (void)hipFree(b->d_tasks);
        b->d_tasks = nullptr;
        b->tasks_cap = 0;
        if ((e = hipMalloc(&b->d_tasks, t.size() * sizeof(int))) != hipSuccess)
            return fail(GS_ERR_OUT_OF_MEMORY, "hipMalloc(batch tasks) failed");
        b->tasks_cap = t.size();
    }
    if ((e = hipMemcpy(b->d_tasks, t.data(), t.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(batch tasks)");
    b->ntasks = (int)(t.size() / gsk::BATCH_TASK_INTS);
    b->tasks_mult = mult;
    b->tasks_lf = lf;
    b->tasks_queue = queue;
    return GS_OK;
}

// Descriptors (they carry the rho / u pointers) to device memory when they changed.
gs_status upload_probs(gs_batch_s* b, const std::vector<gsk::BatchMember>& m) {
    std::vector<unsigned char> bytes;
    gsk::batch_problems(m, bytes);
    if (bytes == b->probs_dev) return GS_OK;
    hipError_t e = hipSuccess;
    if (b->staged_pending && (e = hipEventSynchronize(b->ev_staged)) != hipSuccess)
        return hip_fail(e, "batch staging");
    std::memcpy(b->h_stage, bytes.data(), bytes.size());
    if ((e = hipMemcpyAsync(b->d_probs, b->h_stage, bytes.size(), hipMemcpyHostToDevice, b->own)) != hipSuccess ||
        (e = hipEventRecord(b->ev_staged, b->own)) != hipSuccess)
        return hip_fail(e, "batch descriptor upload");
    b->staged_pending = true;
    b->probs_dev.swap(bytes);
    return GS_OK;
}

// Queues one evaluation of the whole batch on the batch stream under cfg.
// Persistent grid of a launch under c.  With per-die queues every die must run blocks of
// the launch, or the queues of the dies without any are never drained: the grid is then
// at least the co-resident block count (blocks of a full co-resident grid land on every
// die).
int launch_grid(const gs_batch_s* b, const TuneEntry& c) {
    const int grid = c.grid > 0 ? c.grid : b->resident;
    if (c.schedule == GS_SCHED_QUEUE && b->queues.local) return std::max(grid, b->resident);
    return grid;
}

// Creates the side streams on first use (default priority, non-blocking) and forks them from
// the batch stream: work queued on them after this runs after everything queued on `own`.
hipError_t fork_side(gs_batch_s* b) {
    hipError_t e = hipSuccess;
    if (b->side.empty()) {
        b->side.assign(kSideStreams, nullptr);
        b->side_done.assign(kSideStreams, nullptr);
        for (int i = 0; i < kSideStreams && e == hipSuccess; ++i)
            e = hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking);
        for (int i = 0; i < kSideStreams && e == hipSuccess; ++i)
            e = hipEventCreateWithFlags(&b->side_done[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    if ((e = hipEventRecord(b->ev_fork, b->own)) != hipSuccess) return e;
    for (hipStream_t st : b->side)
        if ((e = hipStreamWaitEvent(st, b->ev_fork, 0)) != hipSuccess) return e;
    return hipSuccess;
}

// Joins the side streams back into the batch stream.
hipError_t join_side(gs_batch_s* b) {
    hipError_t e = hipSuccess;
    for (int i = 0; i < kSideStreams && e == hipSuccess; ++i) {
        if ((e = hipEventRecord(b->side_done[i], b->side[i])) == hipSuccess)
            e = hipStreamWaitEvent(b->own, b->side_done[i], 0);
    }
    return e;
}

// GS_SCHED_CONCURRENT: the sized launches of each grid size, in pass order, on side stream
// (size class index mod kSideStreams).
hipError_t launch_concurrent(gs_batch_s* b) {
    hipError_t e = fork_side(b);
    if (e != hipSuccess) return e;
    std::vector<int> sizes;                         // size classes in order of appearance
    for (size_t i = 0; i + 3 < b->runs.size(); i += 4)
        if (std::find(sizes.begin(), sizes.end(), b->runs[i + 1]) == sizes.end()) sizes.push_back(b->runs[i + 1]);
    for (size_t c = 0; c < sizes.size() && e == hipSuccess; ++c) {
        std::vector<int> mine;
        for (size_t i = 0; i + 3 < b->runs.size(); i += 4)
            if (b->runs[i + 1] == sizes[c]) mine.insert(mine.end(), b->runs.begin() + i, b->runs.begin() + i + 4);
        e = gsk::launch_batch_sized(b->d_probs, b->d_tasks, mine, b->side[c % kSideStreams]);
    }
    const hipError_t j = join_side(b);
    return e != hipSuccess ? e : j;
}

// GS_SCHED_STREAMS: each plan's own evaluation launches, the plans (largest first) dealt
// round-robin to the side streams.
gs_status launch_streams(gs_batch_s* b, const double* const* rho, double* const* u) {
    hipError_t e = fork_side(b);
    if (e != hipSuccess) return hip_fail(e, "batch stream fork");
    std::vector<int> order(b->plans.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    auto pts = [&](int i) {
        const gs_plan p = b->plans[i];
        return (double)p->nc[0] * p->nc[1] * (p->d == 3 ? p->nc[2] : 1);
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return pts(x) > pts(y); });
    gs_status st = GS_OK;
    for (size_t k = 0; k < order.size() && st == GS_OK; ++k) {
        const int i = order[k];
        gs_plan p = b->plans[i];
        const hipStream_t keep = p->stream;
        p->stream = b->side[k % kSideStreams];
        st = eval_chain(p, rho[i], u[i], -1);
        p->stream = keep;
    }
    e = join_side(b);
    if (st != GS_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "batch stream join");
    return GS_OK;
}

gs_status launch(gs_batch_s* b, const TuneEntry& c, const double* const* rho, double* const* u) {
    hipError_t e = hipSuccess;
    const int grid = launch_grid(b, c);
    if (c.schedule == GS_SCHED_STREAMS) return launch_streams(b, rho, u);
    if (c.schedule == GS_SCHED_QUEUE) {
        e = gsk::launch_batch_queue(b->d_probs, b->d_tasks, b->queues, b->d_ctr, b->nctr, grid, kSpinLimit, b->own);
    } else if (c.schedule == GS_SCHED_PHASED) {
        e = gsk::launch_batch_phased(b->d_probs, b->d_tasks, b->pass_off, b->pass_cnt, grid, b->own);
    } else if (c.schedule == GS_SCHED_SIZED) {
        e = gsk::launch_batch_sized(b->d_probs, b->d_tasks, b->runs, b->own);
    } else if (c.schedule == GS_SCHED_CONCURRENT) {
        e = launch_concurrent(b);
    } else {
        for (size_t i = 0; i < b->plans.size(); ++i) {
            gs_plan p = b->plans[i];
            const hipStream_t keep = p->stream;
            p->stream = b->own;
            const gs_status st = eval_chain(p, rho[i], u[i], -1);
            p->stream = keep;
            if (st != GS_OK) return st;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return GS_OK;
}

std::string shape_key(const gs_batch_s* b) {
    std::map<std::string, int> c;
    for (gs_plan p : b->plans)
    {
        std::string dims = std::to_string(p->nc[0]);
        for (int i = 1; i < p->d; ++i) dims += "x" + std::to_string(p->nc[i]);
        c[std::to_string(p->d) + "d" + dims + (p->kernel == GS_DIPOLAR_3D ? "dip" : "")]++;
    }
    std::string k;
    for (const auto& [s, cnt] : c) k += (k.empty() ? "" : ",") + s + "x" + std::to_string(cnt);
    return k;
}

gs_status time_candidate(gs_batch_s* b, const std::vector<gsk::BatchMember>& m, const TuneEntry& c,
                         const double* const* rho, double* const* u, double& ms) {
    if (!own_launches(c.schedule)) {
        const gs_status st = upload_tasks(b, m, c.tiles_per_task, c.largest_first, c.schedule);
        if (st != GS_OK) return st;
    }
    // a batch that replays a graph times each candidate as a graph replay (launch costs
    // differ most between the schedules there)
    hipGraphExec_t ex = nullptr;
    if (b->req.use_graph) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        const gs_status cst = launch(b, c, rho, u);
        e = hipStreamEndCapture(b->own, &g);
        if (cst != GS_OK) {
            if (g) (void)hipGraphDestroy(g);
            return cst;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    }
    auto run = [&]() -> gs_status {
        if (!ex) return launch(b, c, rho, u);
        const hipError_t e = hipGraphLaunch(ex, b->own);
        return e == hipSuccess ? GS_OK : hip_fail(e, "hipGraphLaunch");
    };
    hipEvent_t t0 = nullptr, t1 = nullptr;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    gs_status st = run();                         // warm-up
    ms = 1e300;
    for (int r = 0; r < 3 && st == GS_OK; ++r) {
        (void)hipEventRecord(t0, b->own);
        st = run();
        (void)hipEventRecord(t1, b->own);
        const hipError_t e = hipEventSynchronize(t1);
        if (e != hipSuccess) st = hip_fail(e, "autotune timing");
        float f = 0.f;
        (void)hipEventElapsedTime(&f, t0, t1);
        ms = std::min(ms, (double)f);
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (ex) {
        (void)hipStreamSynchronize(b->own);
        (void)hipGraphExecDestroy(ex);
    }
    return st;
}

gs_status autotune(gs_batch_s* b, const std::vector<gsk::BatchMember>& m, const double* const* rho,
                   double* const* u) {
    const std::string key = tune_device_key(b->device) + "|batch|" + shape_key(b) + (b->req.use_graph ? "|graph" : "");
    TuneEntry best;
    if (tune_lookup(key, best) && (own_launches(best.schedule) || b->kernels_ok)) {
        b->cfg = best;
        b->autotuned = true;
        b->tuned_ms = best.ms;
        log(1, "batch autotune (cached): schedule %d, %d tiles per task, %.4f ms", best.schedule,
            best.tiles_per_task, best.ms);
        return GS_OK;
    }
    std::vector<TuneEntry> cand;
    if (b->kernels_ok) {
        for (int mult : {4, 8, 16, 64}) cand.push_back({GS_SCHED_QUEUE, mult, 1, 0, 0.0});
        for (int mult : {1, 2, 4, 16}) cand.push_back({GS_SCHED_PHASED, mult, 1, 0, 0.0});
        for (int mult : {1, 4}) cand.push_back({GS_SCHED_SIZED, mult, 1, 0, 0.0});
        for (int mult : {1, 4}) cand.push_back({GS_SCHED_CONCURRENT, mult, 1, 0, 0.0});
    }
    cand.push_back({GS_SCHED_SEQUENTIAL, 1, 1, 0, 0.0});
    cand.push_back({GS_SCHED_STREAMS, 1, 1, 0, 0.0});
    best.ms = 1e300;
    for (TuneEntry c : cand) {
        double ms = 0.0;
        const gs_status st = time_candidate(b, m, c, rho, u, ms);
        if (st != GS_OK) return st;
        b->candidates++;
        if (ms < best.ms) {
            best = c;
            best.ms = ms;
        }
    }
    tune_store(key, best);
    b->cfg = best;
    b->autotuned = true;
    b->tuned_ms = best.ms;
    log(1, "batch autotune: schedule %d, %d tiles per task, %.4f ms (%zu candidates timed)", best.schedule,
        best.tiles_per_task, best.ms, cand.size());
    return GS_OK;
}

}  // namespace

extern "C" {

void gs_batch_options_default(gs_batch_options* opt) {
    if (opt) std::memset(opt, 0, sizeof(*opt));
}

gs_status gs_batch_create(gs_batch* out, int count, const gs_plan* plans, const gs_batch_options* opt_in) {
    if (!out) return fail(GS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    gs_batch_options opt;
    gs_batch_options_default(&opt);
    if (opt_in) opt = *opt_in;
    if (count < 1 || !plans) return fail(GS_ERR_INVALID_ARG, "invalid batch arguments");
    if (opt.schedule < GS_SCHED_AUTO || opt.schedule > GS_SCHED_STREAMS || opt.tiles_per_task < 0 || opt.grid < 0)
        return fail(GS_ERR_INVALID_ARG, "invalid batch options");
    std::unordered_set<gs_plan> seen;
    bool kernels_ok = true;
    for (int i = 0; i < count; ++i) {
        gs_plan p = plans[i];
        if (!is_live(p) || p->host_only) return fail(GS_ERR_INVALID_ARG, "invalid plan in batch");
        if (!p->X1) return fail(GS_ERR_INVALID_ARG, "a batched plan needs its workspace (GS_PLAN_NO_WORKSPACE)");
        if (!seen.insert(p).second) return fail(GS_ERR_INVALID_ARG, "a plan appears twice in the batch");
        if (p->device != plans[0]->device) return fail(GS_ERR_INVALID_ARG, "batch spans devices");
        if (!p->cube || p->pad != 2 || !gsk::batch_size_supported(p->d, p->n)) {
            if (opt.schedule == GS_SCHED_QUEUE || opt.schedule == GS_SCHED_PHASED || opt.schedule == GS_SCHED_SIZED ||
                opt.schedule == GS_SCHED_CONCURRENT)
                return fail(GS_ERR_UNSUPPORTED_SIZE,
                            "batched kernels cover grids padded to twice their box with the same n <= 128 of "
                            "the compiled list on every axis");
            kernels_ok = false;
        }
        if (p->nslabs != 1) {
            if (opt.schedule == GS_SCHED_QUEUE || opt.schedule == GS_SCHED_PHASED || opt.schedule == GS_SCHED_SIZED ||
                opt.schedule == GS_SCHED_CONCURRENT)
                return fail(GS_ERR_INVALID_ARG, "a batched plan must run its middle passes in one slab");
            kernels_ok = false;
        }
        // the batched kernels run the default radix plans: a plan on a variant (which rounds
        // differently) keeps the schedules that run its own launches
        if (p->cube && (p->tile_bits & (31 << 8))) {
            if (opt.schedule == GS_SCHED_QUEUE || opt.schedule == GS_SCHED_PHASED || opt.schedule == GS_SCHED_SIZED ||
                opt.schedule == GS_SCHED_CONCURRENT)
                return fail(GS_ERR_INVALID_ARG,
                            "a plan on a radix-plan variant is batched by its own launches only "
                            "(sequential or streams schedule)");
            kernels_ok = false;
        }
    }
    auto* b = new gs_batch_s();
    b->plans.assign(plans, plans + count);
    b->device = plans[0]->device;
    b->user = (hipStream_t)opt.stream;
    b->req = opt;
    b->kernels_ok = kernels_ok;
    for (gs_plan p : b->plans) b->points += (double)p->nc[0] * p->nc[1] * (p->d == 3 ? p->nc[2] : 1);
    DeviceScope ds(b->device);
    hipError_t e = ds.err;
    gs_status st = GS_OK;
    std::vector<gsk::BatchMember> m;
    {
        std::vector<const double*> r(count, nullptr);
        std::vector<double*> w(count, nullptr);
        std::vector<double> dummy(1);
        for (int i = 0; i < count; ++i) {
            r[i] = dummy.data();
            w[i] = dummy.data();
        }
        st = members(b, r.data(), w.data(), m);
    }
    std::vector<unsigned char> bytes;
    gsk::batch_problems(m, bytes);
    b->probs_bytes = bytes.size();
    b->nctr = gsk::batch_counters(count);
    if (st == GS_OK && e != hipSuccess) st = hip_fail(e, "hipSetDevice");
    if (st == GS_OK && (e = hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking)) != hipSuccess)
        st = hip_fail(e, "hipStreamCreate");
    if (st == GS_OK && ((e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming)) != hipSuccess ||
                        (e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming)) != hipSuccess ||
                        (e = hipEventCreateWithFlags(&b->ev_staged, hipEventDisableTiming)) != hipSuccess))
        st = hip_fail(e, "hipEventCreate");
    if (st == GS_OK && (hipMalloc(&b->d_probs, b->probs_bytes) != hipSuccess ||
                        hipMalloc(&b->d_ctr, (b->nctr + 1) * sizeof(unsigned)) != hipSuccess ||
                        hipHostMalloc(&b->h_stage, b->probs_bytes) != hipSuccess ||
                        hipHostMalloc(&b->h_flag, sizeof(unsigned)) != hipSuccess))
        st = fail(GS_ERR_OUT_OF_MEMORY, "batch allocation failed");
    if (st == GS_OK) *b->h_flag = 0u;
    if (st == GS_OK) {
        // the queue counters and the error flag start at zero; each queue launch
        // leaves the counters at zero
        std::vector<unsigned> zero(b->nctr + 1, 0u);
        if ((e = hipMemcpy(b->d_ctr, zero.data(), zero.size() * sizeof(unsigned), hipMemcpyHostToDevice)) !=
            hipSuccess)
            st = hip_fail(e, "hipMemcpy(batch counters)");
    }
    if (st == GS_OK) b->resident = gsk::batch_resident_blocks();
    if (st == GS_OK && opt.schedule != GS_SCHED_AUTO) {
        // default task sizes: the queue schedule pays an agent-scope release and
        // acquire per task, so its tasks are larger
        const int def = opt.schedule == GS_SCHED_QUEUE ? kQueueTilesPerTask : 4;
        b->cfg = {opt.schedule, opt.tiles_per_task > 0 ? opt.tiles_per_task : def, 1, opt.grid, 0.0};
        if (!own_launches(opt.schedule)) st = upload_tasks(b, m, b->cfg.tiles_per_task, 1, opt.schedule);
        b->resolved = true;
    }
    if (st != GS_OK) {
        (void)hipGetLastError();
        release(b);
        return st;
    }
    std::lock_guard<std::mutex> g(g_batch_mu);
    g_batches.insert(b);
    *out = b;
    return GS_OK;
}

gs_status gs_batch_eval(gs_batch b, const double* const* rho, double* const* u) {
    if (!batch_live(b)) return fail(GS_ERR_INVALID_ARG, "invalid batch");
    if (!rho || !u) return fail(GS_ERR_INVALID_ARG, "NULL pointer array");
    for (size_t i = 0; i < b->plans.size(); ++i) {
        if (!is_live(b->plans[i])) return fail(GS_ERR_INVALID_ARG, "a plan of the batch was destroyed");
        if (!rho[i] || !u[i]) return fail(GS_ERR_INVALID_ARG, "NULL device pointer in batch");
    }
    // the error flag of an earlier queue launch, as far as its copy has arrived (the flag
    // is sticky: once a launch raised it, every later check sees it)
    if (*reinterpret_cast<volatile unsigned*>(b->h_flag))
        return fail(GS_ERR_HIP, "an earlier queue-schedule evaluation of this batch left tasks unfinished "
                                "(its results are invalid)");
    DeviceScope ds(b->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    std::vector<gsk::BatchMember> m;
    gs_status st = members(b, rho, u, m);
    if (st != GS_OK) return st;
    hipError_t e;
    if ((e = hipEventRecord(b->ev_in, b->user)) != hipSuccess || (e = hipStreamWaitEvent(b->own, b->ev_in, 0)) != hipSuccess)
        return hip_fail(e, "batch stream ordering");
    if ((st = upload_probs(b, m)) != GS_OK) return st;
    if (!b->resolved) {
        if ((st = autotune(b, m, rho, u)) != GS_OK) return st;
        b->resolved = true;
    }
    if (!own_launches(b->cfg.schedule) &&
        (st = upload_tasks(b, m, b->cfg.tiles_per_task, b->cfg.largest_first, b->cfg.schedule)) != GS_OK)
        return st;
    if (b->req.use_graph) {
        // what the captured launches bake in: the task list, and for the sequential
        // schedule the rho / u pointers themselves
        std::vector<const void*> sig = {b->d_tasks, (const void*)(intptr_t)b->ntasks,
                                        (const void*)(intptr_t)b->cfg.schedule};
        if (own_launches(b->cfg.schedule))
            for (size_t i = 0; i < b->plans.size(); ++i) {
                sig.push_back(rho[i]);
                sig.push_back(u[i]);
            }
        if (!b->exec || sig != b->graph_sig) {
            if (b->exec) {
                (void)hipStreamSynchronize(b->own);
                (void)hipGraphExecDestroy(b->exec);
                b->exec = nullptr;
            }
            hipGraph_t g = nullptr;
            if ((e = hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return hip_fail(e, "hipStreamBeginCapture");
            st = launch(b, b->cfg, rho, u);
            e = hipStreamEndCapture(b->own, &g);
            if (st != GS_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                b->exec = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
            b->graph_sig = sig;
        }
        if ((e = hipGraphLaunch(b->exec, b->own)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
        if ((st = launch(b, b->cfg, rho, u)) != GS_OK) return st;
    }
    if (b->cfg.schedule == GS_SCHED_QUEUE &&
        (e = hipMemcpyAsync(b->h_flag, b->d_ctr + b->nctr, sizeof(unsigned), hipMemcpyDeviceToHost, b->own)) !=
            hipSuccess)
        return hip_fail(e, "batch error flag copy");
    if ((e = hipEventRecord(b->ev_out, b->own)) != hipSuccess || (e = hipStreamWaitEvent(b->user, b->ev_out, 0)) != hipSuccess)
        return hip_fail(e, "batch stream ordering");
    return GS_OK;
}

gs_status gs_batch_query(gs_batch b, gs_batch_info* info) {
    if (!batch_live(b) || !info) return fail(GS_ERR_INVALID_ARG, "invalid batch or info");
    std::memset(info, 0, sizeof(*info));
    info->count = (int)b->plans.size();
    info->points = b->points;
    info->schedule = b->resolved ? b->cfg.schedule : GS_SCHED_AUTO;
    info->tiles_per_task = b->cfg.tiles_per_task;
    info->grid = launch_grid(b, b->cfg);
    info->use_graph = b->req.use_graph;
    info->num_tasks = b->ntasks;
    for (int p = 0; p < 6; ++p) info->tasks_per_pass[p] = b->pass_cnt[p];
    info->autotuned = b->autotuned ? 1 : 0;
    info->candidates = b->candidates;
    info->tuned_ms = b->tuned_ms;
    DeviceScope ds(b->device);
    unsigned flag = 0;
    hipError_t e = hipStreamSynchronize(b->own);
    if (e == hipSuccess)
        e = hipMemcpy(&flag, b->d_ctr + b->nctr, sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "batch query");
    info->wait_timeouts = flag ? 1 : 0;
    info->num_queues = b->queues.nq;
    info->local_queues = b->queues.local;
    return GS_OK;
}

gs_status gs_batch_destroy(gs_batch b) {
    if (!b) return GS_OK;
    {
        std::lock_guard<std::mutex> g(g_batch_mu);
        if (!g_batches.count(b)) return GS_OK;
        g_batches.erase(b);
    }
    release(b);
    return GS_OK;
}

gs_status gs_eval_batch(int count, const gs_plan* plans, const double* const* rho_dev, double* const* u_dev) {
    if (count <= 0 || !plans || !rho_dev || !u_dev) return fail(GS_ERR_INVALID_ARG, "invalid batch arguments");
    for (int i = 0; i < count; ++i)
        if (!is_live(plans[i])) return fail(GS_ERR_INVALID_ARG, "invalid plan in batch");
    gs_batch_options opt;
    gs_batch_options_default(&opt);
    opt.schedule = GS_SCHED_QUEUE;
    opt.stream = plans[0]->stream;
    gs_batch b = nullptr;
    gs_status st = gs_batch_create(&b, count, plans, &opt);
    if (st != GS_OK) return st;
    st = gs_batch_eval(b, rho_dev, u_dev);
    if (st == GS_OK) {
        // waits for the evaluation and reads the error flag
        gs_batch_info info;
        st = gs_batch_query(b, &info);
        if (st == GS_OK && info.wait_timeouts)
            st = fail(GS_ERR_HIP, "batched evaluation left tasks unfinished (results invalid)");
    }
    const gs_status st2 = gs_batch_destroy(b);
    return st != GS_OK ? st : st2;
}

gs_status gs_batch_set_stream(gs_batch b, void* stream) {
    if (!batch_live(b)) return fail(GS_ERR_INVALID_ARG, "invalid batch");
    b->user = (hipStream_t)stream;
    return GS_OK;
}

}  // extern "C"
