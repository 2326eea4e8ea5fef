// batch.hip -- host side of the batched evaluation: descriptors, task lists, launches.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <set>
#include <cstring>
#include <numeric>
#include <vector>

#include "batch.hpp"
#include "device_api.hpp"

namespace gsk {

static_assert(sizeof(BatchTask) == BATCH_TASK_INTS * sizeof(int), "task layout");

bool batch_size_supported(int d, int n) {
    if (d != 2 && d != 3) return false;
    switch (n) {
#define GS_CASE(N) \
    case N: return true;
        GS_BATCH_SIZES(GS_CASE)
#undef GS_CASE
        default: return false;
    }
}

static int threads_for(int n, int pass) {
    switch (n) {
#define GS_CASE(N) \
    case N: return tile_threads<N>(pass);
        GS_BATCH_SIZES(GS_CASE)
#undef GS_CASE
    }
    return 0;
}

static int tiles_for(int n, int pass, int d) {
    switch (n) {
#define GS_CASE(N) \
    case N: return tile_count<N>(pass, d);
        GS_BATCH_SIZES(GS_CASE)
#undef GS_CASE
    }
    return 0;
}

void batch_problems(const std::vector<BatchMember>& m, std::vector<unsigned char>& out) {
    out.assign(m.size() * sizeof(BatchProblem), 0);
    for (size_t b = 0; b < m.size(); ++b) {
        const BatchMember& a = m[b];
        BatchProblem P;
        P.n = a.n;
        P.d = a.d;
        P.mode = a.dipolar ? SPEC_DIPOLAR : SPEC_PLAIN;
        P.rho = a.rho;
        P.u = a.u;
        P.X1 = reinterpret_cast<cpx*>(a.X1);
        P.X2 = reinterpret_cast<cpx*>(a.X2);
        P.spec = a.spec;
        P.tw = reinterpret_cast<const cpx*>(a.tw);
        for (int i = 0; i < 3; ++i) P.dip.dxi[i] = a.dxi[i];
        for (int i = 0; i < 3; ++i) {
            P.dip.cdiag[i] = a.cdiag[i];
            P.dip.ccross[i] = a.ccross[i];
        }
        P.dip.nm_over_M = a.nm_over_M;
        std::memcpy(out.data() + b * sizeof(BatchProblem), &P, sizeof(P));
    }
}

// Tasks per pass of one problem below which its tasks are made smaller than the requested size.
constexpr int kMinTasksPerPass = 24;

// Pass-major tasks of the members listed in `order` (indices into m), appended to T.
static void build_tasks(const std::vector<BatchMember>& m, const std::vector<int>& order, int mult,
                        std::vector<BatchTask>& T, int pass_off[6], int pass_cnt[6]) {
    std::vector<int> ntask(m.size() * 6, 0);      // tasks of pass p of member b
    for (int p = 1; p <= 5; ++p) {
        pass_off[p] = (int)T.size();
        for (int b : order) {
            const int d = m[b].d, n = m[b].n;
            if (d == 2 && (p == 2 || p == 4)) continue;
            const int dep = (p == 1) ? 0 : (d == 2 ? p - 2 : p - 1);
            const int per = BATCH_THREADS / threads_for(n, p);     // tiles per block-full
            const int nt = tiles_for(n, p, d);
            // a pass of few block-fulls gets smaller tasks (down to one block-full): at least
            // kMinTasksPerPass of them where it has that many, so that a small problem's pass
            // is not left to a few blocks working through long tasks while the others wait
            const int fulls = (nt + per - 1) / per;
            const int step = per * std::max(1, std::min(std::max(1, mult), fulls / kMinTasksPerPass));
            for (int t = 0; t < nt; t += step) {
                BatchTask k;
                k.prob = b;
                k.pass = p;
                k.tile0 = t;
                k.tile1 = std::min(nt, t + step);
                k.dep_pass = dep;
                k.dep_count = dep ? ntask[b * 6 + dep] : 0;
                T.push_back(k);
                ntask[b * 6 + p]++;
            }
        }
        pass_cnt[p] = (int)T.size() - pass_off[p];
    }
    pass_off[0] = pass_cnt[0] = 0;
}

// Relative cost per grid point of a 3D problem in the batched kernels, by n: measured with the
// phased schedule on batches of one size (ns per point: 32: 0.071, 48: 0.065, 64: 0.046,
// 96: 0.058, 128: 0.048), taken relative to 128; the lengths below 32 extrapolated.  Small and
// radix-3 lengths cost more per point, so weighing problems by their point count alone left
// the die with the most small problems 5 % behind the others.
static double point_cost_3d(int n) {
    switch (n) {
        case 8: return 2.0;
        case 12: return 1.8;
        case 16: return 1.6;
        case 24: return 1.5;
        case 32: return 1.48;
        case 48: return 1.35;
        case 64: return 0.96;
        case 96: return 1.21;
        default: return 1.0;
    }
}

static double member_work(const BatchMember& x) {
    return std::pow((double)x.n, x.d) * (x.d == 3 ? 2.5 * point_cost_3d(x.n) : 1.0);
}

static std::vector<int> size_order(const std::vector<BatchMember>& m, bool largest_first) {
    std::vector<int> order(m.size());
    std::iota(order.begin(), order.end(), 0);
    if (largest_first)
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return member_work(m[a]) > member_work(m[b]); });
    return order;
}

void batch_tasks(const std::vector<BatchMember>& m, int mult, bool largest_first, std::vector<int>& tasks,
                 int pass_off[6], int pass_cnt[6]) {
    std::vector<BatchTask> T;
    build_tasks(m, size_order(m, largest_first), mult, T, pass_off, pass_cnt);
    tasks.resize(T.size() * BATCH_TASK_INTS);
    std::memcpy(tasks.data(), T.data(), T.size() * sizeof(BatchTask));
}

void batch_queue_tasks(const std::vector<BatchMember>& m, int mult, int nq, std::vector<int>& tasks,
                       std::vector<int>& qoff) {
    nq = std::max(1, nq);
    // members dealt to queues by decreasing work, each to the least loaded queue
    std::vector<std::vector<int>> part(nq);
    std::vector<double> load(nq, 0.0);
    for (int b : size_order(m, true)) {
        const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        part[q].push_back(b);
        load[q] += member_work(m[b]);
    }
    std::vector<BatchTask> T;
    qoff.assign(nq + 1, 0);
    for (int q = 0; q < nq; ++q) {
        int off[6], cnt[6];
        build_tasks(m, part[q], mult, T, off, cnt);
        qoff[q + 1] = (int)T.size();
    }
    tasks.resize(T.size() * BATCH_TASK_INTS);
    std::memcpy(tasks.data(), T.data(), T.size() * sizeof(BatchTask));
}

__global__ void k_xcc_probe(int* out) {
    if (threadIdx.x == 0) out[blockIdx.x] = hw_xcc_id();
}

int batch_xcc_ids(int* ids, int cap) {
    static std::mutex mu;
    static std::map<int, std::vector<int>> cache;      // device -> sorted ids
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it == cache.end()) {
        constexpr int NB = 2048;
        int* d = nullptr;
        std::vector<int> h(NB, -1), found;
        if (hipMalloc(&d, NB * sizeof(int)) == hipSuccess) {
            k_xcc_probe<<<NB, 64>>>(d);
            if (hipGetLastError() == hipSuccess &&
                hipMemcpy(h.data(), d, NB * sizeof(int), hipMemcpyDeviceToHost) == hipSuccess) {
                std::set<int> s(h.begin(), h.end());
                found.assign(s.begin(), s.end());
            }
            (void)hipFree(d);
        }
        (void)hipGetLastError();
        it = cache.emplace(dev, found).first;
    }
    const int c = (int)it->second.size();
    for (int i = 0; i < c && i < cap; ++i) ids[i] = it->second[i];
    return c;
}

int batch_counters(int nprob) { return batch_counter(nprob, 0); }

int batch_resident_blocks() {
    int dev = 0, cus = 0, a = 0, b = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, (const void*)k_batch_queue, BATCH_THREADS, 0);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void*)k_batch_pass<3>, BATCH_THREADS, 0);
    const int per = std::max(1, std::min(a > 0 ? a : 1, b > 0 ? b : 1));
    return cus * per;
}

hipError_t launch_batch_queue(const void* probs, const void* tasks, const BatchQueueSpec& spec, unsigned* ctr,
                              int nctr, int grid, unsigned spin_limit, hipStream_t s) {
    if (spec.nq < 1 || spec.nq > BATCH_MAX_QUEUES || (int)spec.qoff.size() != spec.nq + 1) return hipErrorInvalidValue;
    if (spec.qoff[spec.nq] <= 0) return hipSuccess;
    if (grid <= 0) return hipErrorInvalidValue;
    BatchQueues Q;
    Q.nq = spec.nq;
    Q.local = spec.local;
    for (int i = 0; i < BATCH_MAX_QUEUES; ++i) Q.qmap[i] = spec.qmap[i];
    for (int i = 0; i <= BATCH_MAX_QUEUES; ++i) Q.qoff[i] = i <= spec.nq ? spec.qoff[i] : spec.qoff[spec.nq];
    // local queues need blocks on every die: the whole co-resident grid
    const int g = spec.local ? grid : std::min(grid, spec.qoff[spec.nq]);
    k_batch_queue<<<g, BATCH_THREADS, 0, s>>>(static_cast<const BatchProblem*>(probs),
                                               static_cast<const BatchTask*>(tasks), Q, ctr, nctr, spin_limit);
    return hipGetLastError();
}

hipError_t launch_batch_phased(const void* probs, const void* tasks, const int pass_off[6], const int pass_cnt[6],
                               int grid, hipStream_t s) {
    if (grid <= 0) return hipErrorInvalidValue;
    auto P = static_cast<const BatchProblem*>(probs);
    auto T = static_cast<const BatchTask*>(tasks);
    for (int p = 1; p <= 5; ++p) {
        const int c = pass_cnt[p];
        if (c <= 0) continue;
        const int g = std::min(grid, c);
        const BatchTask* tp = T + pass_off[p];
        switch (p) {
            case 1: k_batch_pass<1><<<g, BATCH_THREADS, 0, s>>>(P, tp, c); break;
            case 2: k_batch_pass<2><<<g, BATCH_THREADS, 0, s>>>(P, tp, c); break;
            case 3: k_batch_pass<3><<<g, BATCH_THREADS, 0, s>>>(P, tp, c); break;
            case 4: k_batch_pass<4><<<g, BATCH_THREADS, 0, s>>>(P, tp, c); break;
            case 5: k_batch_pass<5><<<g, BATCH_THREADS, 0, s>>>(P, tp, c); break;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int N, int PASS> static int size_grid() {
    static const int g = [] {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_batch_size<N, PASS>, BATCH_THREADS, 0);
        return cus * (per > 0 ? per : 1);
    }();
    return g;
}

template <int PASS>
static hipError_t launch_size(int n, const BatchProblem* P, const BatchTask* T, int cnt, int mult_grid, hipStream_t s) {
    switch (n) {
#define GS_CASE(N)                                                                            \
    case N: {                                                                                 \
        const int g = std::min(cnt, std::max(1, size_grid<N, PASS>() * mult_grid));          \
        k_batch_size<N, PASS><<<g, BATCH_THREADS, 0, s>>>(P, T, cnt);                         \
        break;                                                                                \
    }
        GS_BATCH_SIZES(GS_CASE)
#undef GS_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_sized(const void* probs, const void* tasks, const std::vector<int>& runs, hipStream_t s) {
    auto P = static_cast<const BatchProblem*>(probs);
    auto T = static_cast<const BatchTask*>(tasks);
    for (size_t i = 0; i + 3 < runs.size(); i += 4) {
        const int pass = runs[i], n = runs[i + 1], off = runs[i + 2], cnt = runs[i + 3];
        hipError_t e = hipSuccess;
        switch (pass) {
            case 1: e = launch_size<1>(n, P, T + off, cnt, 2, s); break;
            case 2: e = launch_size<2>(n, P, T + off, cnt, 2, s); break;
            case 3: e = launch_size<3>(n, P, T + off, cnt, 2, s); break;
            case 4: e = launch_size<4>(n, P, T + off, cnt, 2, s); break;
            case 5: e = launch_size<5>(n, P, T + off, cnt, 2, s); break;
            default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void batch_size_runs(const std::vector<BatchMember>& m, const std::vector<int>& tasks, std::vector<int>& runs) {
    runs.clear();
    const BatchTask* T = reinterpret_cast<const BatchTask*>(tasks.data());
    const int nt = (int)(tasks.size() / BATCH_TASK_INTS);
    for (int k = 0; k < nt;) {
        const int pass = T[k].pass, n = m[T[k].prob].n;
        int j = k;
        while (j < nt && T[j].pass == pass && m[T[j].prob].n == n) ++j;
        runs.push_back(pass);
        runs.push_back(n);
        runs.push_back(k);
        runs.push_back(j - k);
        k = j;
    }
}

}  // namespace gsk
