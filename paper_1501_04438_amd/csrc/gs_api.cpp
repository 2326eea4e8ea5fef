// gs_api.cpp -- the C ABI declared in include/gs.h.
//
// A plan owns the Gaussian-sum table, the factor matrix, the Taylor constants,
// the stored spectrum octant (device), the FFT twiddle table (device) and the
// evaluation workspace (device): X1 = (n+1) n^(d-1) complex values, and in 3D
// X2 = 2n n (n+1) complex values.  Nothing is allocated per evaluation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <utility>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/gs.h"
#include "device_api.hpp"
#include "host_plan.hpp"
#include "api_internal.hpp"
#include "autotune.hpp"
#include "sizes.hpp"


namespace gsapi {

thread_local std::string g_err;
std::mutex g_live_mu;
std::unordered_set<gs_plan_s*> g_live;

gs_status fail(gs_status s, const std::string& msg) {
    g_err = msg;
    log(2, "error %d: %s", (int)s, msg.c_str());
    return s;
}

void log(int level, const char* fmt, ...) {
    const char* env = std::getenv("GS_LOG_LEVEL");
    if (!env || std::atoi(env) < level) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[gs] %s\n", buf);
}

gs_status hip_fail(hipError_t e, const char* what) {
    return fail(GS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool is_live(gs_plan p) {
    std::lock_guard<std::mutex> g(g_live_mu);
    return p && g_live.count(p);
}

}  // namespace gsapi

using namespace gsapi;

namespace {

int visible_devices() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

void free_device(gs_plan_s* p) {
    if (p->host_only) return;
    DeviceScope ds(p->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    else (void)hipDeviceSynchronize();
    if (p->spec) (void)hipFree(p->spec);
    if (p->X1) (void)hipFree(p->X1);
    if (p->X2) (void)hipFree(p->X2);
    if (p->tw) (void)hipFree(p->tw);
    for (int i = 0; i < 3; ++i) {
        bool shared = p->twk[i] == p->tw;
        for (int j = 0; j < i; ++j) shared = shared || p->twk[j] == p->twk[i];
        if (p->twk[i] && !shared) (void)hipFree(p->twk[i]);
        p->twk[i] = nullptr;
    }
    if (p->epart) (void)hipFree(p->epart);
    if (p->mixpart) (void)hipFree(p->mixpart);
    if (p->E) (void)hipFree(p->E);
    p->epart = p->mixpart = p->E = nullptr;
    for (hipStream_t st : p->sstreams) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : p->sevents) (void)hipEventDestroy(ev);
    p->sstreams.clear();
    p->sevents.clear();
    p->spec = nullptr;
    p->X1 = p->X2 = p->tw = nullptr;
}

gs_status device_assembly(gs_plan_s* p) {
    const int Q = (int)p->table.w.size();
    const int n1 = p->nk[0] + 1, n1b = p->nk[1] + 1, n1c = p->nk[p->d - 1] + 1;
    const int Qp = (Q + 3) / 4 * 4;
    const int ldk = std::max(gsk::assembly_ldk(n1), std::max(n1b, n1c));
    const size_t sz = (size_t)Qp * ldk;
    // operands [Qp][ldk], transposed factors: w_q Fx (AT), then Fy, then (3D) Fz
    const int nf = p->d - 1;                   // factor blocks after AT: y (and z)
    std::vector<double> ops(sz * (1 + nf), 0.0);
    for (int q = 0; q < Q; ++q) {
        for (int k = 0; k < n1; ++k) ops[(size_t)q * ldk + k] = p->table.w[q] * p->Fk[0][(size_t)k * Q + q];
        for (int j = 1; j <= nf; ++j)
            for (int k = 0; k <= p->nk[j]; ++k) ops[sz * j + (size_t)q * ldk + k] = p->Fk[j][(size_t)k * Q + q];
    }
    double* dops = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&dops, ops.size() * 8)) != hipSuccess) return hip_fail(e, "hipMalloc(assembly)");
    gs_status st = GS_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    do {
        if ((e = hipMemcpyAsync(dops, ops.data(), ops.size() * 8, hipMemcpyHostToDevice, p->stream)) != hipSuccess) {
            st = hip_fail(e, "hipMemcpy(assembly)");
            break;
        }
        gsk::AssemblyArgs a;
        a.d = p->d;
        a.n1 = n1;
        a.n1b = p->d == 3 ? n1b : 0;
        a.n1c = n1c;
        a.Qp = Qp;
        a.ldk = ldk;
        a.AT = dops;
        a.FB = dops + sz;                          // Fy
        a.FC = dops + sz * nf;                     // Fz (3D), Fy (2D)
        a.out = p->spec;
        a.A0 = p->A0;
        a.c2 = p->c2;
        a.dxi[0] = M_PI / (2.0 * p->Lk[0]);
        a.dxi[1] = M_PI / (2.0 * p->Lk[1]);
        a.dxi[2] = M_PI / (2.0 * p->Lk[p->d - 1]);
        double M = 1.0;
        for (int j = 0; j < p->d; ++j) M *= 2.0 * p->nk[j];
        a.invM = 1.0 / M;
        a.dxx = p->kernel == GS_DAVEY_STEWARTSON_2D ? 1 : 0;
        a.lapu = (p->flags & GS_PLAN_UNPADDED_LAPLACIAN) ? p->pad : 0;
        if ((e = gsk::load_assembly(a)) != hipSuccess) {
            st = hip_fail(e, "spectrum assembly kernel load");
            break;
        }
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)hipEventRecord(e0, p->stream);
        if ((e = gsk::launch_assembly(a, p->stream)) != hipSuccess) {
            st = hip_fail(e, "spectrum assembly launch");
            break;
        }
        (void)hipEventRecord(e1, p->stream);
        if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) {
            st = hip_fail(e, "spectrum assembly");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        p->assembly_ms = ms;
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(dops);
    return st;
}

// X2 slab budget in bytes: GS_SLAB_BYTES, else unbounded (one slab).  Measured on
// MI355X at n = 256, slabs sized to the Infinity Cache did not speed the middle
// passes up (X2 written by one pass is not served from it to the next), so slabs
// are a memory cap: X2 shrinks to one slab.
size_t slab_budget() {
    const char* s = std::getenv("GS_SLAB_BYTES");
    if (s && *s) return std::max<size_t>(1, (size_t)std::strtoull(s, nullptr, 10));
    return (size_t)-1;
}

size_t workspace_cap() {
    const char* s = std::getenv("GS_MAX_WORKSPACE_BYTES");
    if (!s || !*s) return (size_t)-1;
    return (size_t)std::strtoull(s, nullptr, 10);
}

gs_status plan_autotune(gs_plan_s* p);

}  // namespace

namespace gsapi {

gs_status make_args(gs_plan p, const double* in, double* out, gsk::EvalArgs& a) {
    if (!is_live(p)) return fail(GS_ERR_INVALID_ARG, "invalid plan");
    if (p->host_only) return fail(GS_ERR_INVALID_ARG, "host-only plan cannot evaluate");
    if (!in || !out) return fail(GS_ERR_INVALID_ARG, "NULL device pointer");
    a.d = p->d;
    a.n = p->nf;
    a.nx = p->nk[0];
    a.ny = p->nk[1];
    a.nz = p->d == 3 ? p->nk[2] : 1;
    a.twx = p->twk[0];
    a.twy = p->twk[1];
    a.twz = p->d == 3 ? p->twk[2] : nullptr;
    a.rho = in;
    a.u = out;
    if (p->pad == 3) {
        a.pad_in = in;
        a.pad_out = out;
        a.px = p->nu[0];
        a.py = p->nu[1];
        a.pz = p->d == 3 ? p->nu[2] : 1;
        if (p->cube) {
            // the x passes read the density and write the potential at their own extents
            a.emb = 1;
        } else {
            a.rho = p->E;
            a.u = p->E;
        }
    }
    a.X1 = p->X1;
    a.X2 = p->X2;
    a.spec = p->spec;
    a.tw = p->tw;
    for (int i = 0; i < 3; ++i) a.dxi[i] = p->Lk[i] > 0.0 ? M_PI / (2.0 * p->Lk[i]) : 0.0;
    a.hint_bits = p->hint_bits;
    a.fused_grid_mult = p->fused_mult;
    a.tile_bits = p->cube ? p->tile_bits : 0;
    if (p->kernel == GS_DIPOLAR_3D) {
        a.dipolar = 1;
        for (int i = 0; i < 3; ++i) a.cdiag[i] = 3.0 * p->dn[i] * p->dm[i];
        a.ccross[0] = 3.0 * (p->dn[0] * p->dm[1] + p->dn[1] * p->dm[0]);
        a.ccross[1] = 3.0 * (p->dn[0] * p->dm[2] + p->dn[2] * p->dm[0]);
        a.ccross[2] = 3.0 * (p->dn[1] * p->dm[2] + p->dn[2] * p->dm[1]);
        const double nm = p->dn[0] * p->dm[0] + p->dn[1] * p->dm[1] + p->dn[2] * p->dm[2];
        a.nm_over_M = nm / (8.0 * p->nk[0] * p->nk[1] * p->nk[2]);
    }
    return GS_OK;
}

bool set_slabs(gs_plan p, int planes, int streams) {
    if (p->d != 3) return planes >= p->nk[0] + 1 && streams <= 1;
    const int n1 = p->nk[0] + 1;
    planes = std::max(1, std::min(planes, n1));
    const int nsl = (n1 + planes - 1) / planes;
    const int slab = (n1 + nsl - 1) / nsl;
    streams = std::max(1, std::min(streams, nsl));
    if (slab > p->x2_planes || (streams > 1 && p->x2_planes < n1)) return false;
    p->nslabs = nsl;
    p->slab = slab;
    p->nstreams = streams;
    p->steps.clear();
    p->steps.push_back({1, 0});
    for (int c = 0; c < nsl; ++c) {
        p->steps.push_back({2, c});
        p->steps.push_back({3, c});
        p->steps.push_back({4, c});
    }
    p->steps.push_back({5, 0});
    return true;
}

static hipError_t run_step(gs_plan p, gsk::EvalArgs& a, int step, hipStream_t s) {
    const auto [pass, c] = p->steps[step];
    a.kx0 = c * p->slab;
    a.kxn = std::min(p->slab, p->nk[0] + 1 - a.kx0);
    gsk::EvalArgs b = a;
    // X2 holding every plane: the slab's planes sit at its own offset
    if (p->d == 3 && p->x2_planes == p->nk[0] + 1 && p->nslabs > 1)
        b.X2 = a.X2 + (size_t)a.kx0 * 2 * p->nk[1] * p->nk[2];
    const int nz = p->d == 3 ? p->nk[2] : 1;
    hipError_t e = hipSuccess;
    // padding 3: the density into the transform grid before the first step
    // (cubic transform grids: the x passes read and write the caller's arrays themselves)
    if (p->pad == 3 && !a.emb && step == 0)
        e = gsk::launch_pad_embed(a.pad_in, a.u, a.px, a.py, a.pz, p->nk[0], p->nk[1], nz, s);
    if (e == hipSuccess) e = gsk::launch_eval(b, s, pass);
    // and the potential out of it after the last
    if (e == hipSuccess && p->pad == 3 && !a.emb && step == (int)p->steps.size() - 1)
        e = gsk::launch_pad_crop(a.u, a.pad_out, a.px, a.py, a.pz, p->nk[0], p->nk[1], nz, s);
    return e;
}

// The slab chains (y-forward, fused, y-inverse of one kx slab) on p->nstreams streams:
// forked from the plan's stream after the x pass, joined before the x-inverse pass.
static hipError_t run_concurrent(gs_plan p, gsk::EvalArgs& a) {
    const int k = p->nstreams;
    hipError_t e = hipSuccess;
    if ((int)p->sstreams.size() < k) {
        for (hipStream_t st : p->sstreams) (void)hipStreamDestroy(st);
        for (hipEvent_t ev : p->sevents) (void)hipEventDestroy(ev);
        p->sstreams.assign(k, nullptr);
        p->sevents.assign(k + 1, nullptr);
        for (int i = 0; i < k && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&p->sstreams[i], hipStreamNonBlocking);
        for (int i = 0; i <= k && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&p->sevents[i], hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    const int last = (int)p->steps.size() - 1;
    if ((e = run_step(p, a, 0, p->stream)) != hipSuccess) return e;
    if ((e = hipEventRecord(p->sevents[k], p->stream)) != hipSuccess) return e;
    for (int i = 0; i < k; ++i)
        if ((e = hipStreamWaitEvent(p->sstreams[i], p->sevents[k], 0)) != hipSuccess) return e;
    for (int c = 0; c < p->nslabs; ++c) {
        hipStream_t s = p->sstreams[c % k];
        for (int j = 0; j < 3; ++j)
            if ((e = run_step(p, a, 1 + 3 * c + j, s)) != hipSuccess) return e;
    }
    for (int i = 0; i < k; ++i) {
        if ((e = hipEventRecord(p->sevents[i], p->sstreams[i])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(p->stream, p->sevents[i], 0)) != hipSuccess) return e;
    }
    return run_step(p, a, last, p->stream);
}

gs_status eval_chain(gs_plan p, const double* in, double* out, int step, double* energy, bool gradient) {
    gsk::EvalArgs a;
    gs_status st = make_args(p, in, out, a);
    if (st != GS_OK) return st;
    if (energy) {
        a.energy = energy;
        a.epart = p->epart;
        a.epencils = gsk::energy_pencils(p->d, a.nx, a.ny);
        double cell = 1.0;
        for (int i = 0; i < p->d; ++i) cell *= 2.0 * p->Lc[i] / p->nc[i];
        // the energy 1/2 cell sum rho u (the fused pass sums rho u); with gradient the outputs
        // are cell u, its rho gradient
        a.escale = 0.5 * cell;
        a.oscale = gradient ? cell : 1.0;
    }
    if (!p->X1) return fail(GS_ERR_INVALID_ARG, "plan created without a workspace (GS_PLAN_NO_WORKSPACE): "
                                                  "evaluate it with gs_eval_static");
    if (step >= (int)p->steps.size()) return fail(GS_ERR_INVALID_ARG, "step out of range");
    DeviceScope ds(p->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    hipError_t e = hipSuccess;
    if (step >= 0) {
        e = run_step(p, a, step, p->stream);
    } else if (p->d == 3 && p->nstreams > 1 && p->nslabs > 1) {
        e = run_concurrent(p, a);
    } else {
        for (int i = 0; i < (int)p->steps.size() && e == hipSuccess; ++i) e = run_step(p, a, i, p->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "evaluation launch");
    return GS_OK;
}

// X1, X2 and (padding 3) E in complex values
static void workspace_parts(gs_plan p, size_t& x1, size_t& x2, size_t& e) {
    const size_t nx = p->nk[0], ny = p->nk[1], nz = p->d == 3 ? p->nk[2] : 1;
    x1 = (nx + 1) * ny * nz;
    x2 = p->d == 3 ? 2 * ny * nz * (size_t)p->x2_planes : 0;
    e = p->pad == 3 ? (nx * ny * nz + 1) / 2 : 0;
}

size_t workspace_complex(gs_plan p) {
    size_t x1, x2, e;
    workspace_parts(p, x1, x2, e);
    return x1 + x2 + e;
}

gs_status eval_chain_ws(gs_plan p, const double* in, double* out, double2* ws) {
    gsk::EvalArgs a;
    gs_status st = make_args(p, in, out, a);
    if (st != GS_OK) return st;
    size_t x1, x2, ne;
    workspace_parts(p, x1, x2, ne);
    a.X1 = ws;
    a.X2 = p->d == 3 ? ws + x1 : nullptr;
    if (p->pad == 3 && !a.emb) {
        a.rho = reinterpret_cast<const double*>(ws + x1 + x2);
        a.u = reinterpret_cast<double*>(ws + x1 + x2);
    }
    DeviceScope ds(p->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    hipError_t e = hipSuccess;
    for (int i = 0; i < (int)p->steps.size() && e == hipSuccess; ++i) e = run_step(p, a, i, p->stream);
    if (e != hipSuccess) return hip_fail(e, "evaluation launch");
    return GS_OK;
}

}  // namespace gsapi

extern "C" {

void gs_options_default(gs_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->delta_rel = 1e-4;
    opt->device = -1;
}

const char* gs_status_string(gs_status s) {
    switch (s) {
        case GS_OK: return "GS_OK";
        case GS_ERR_INVALID_ARG: return "GS_ERR_INVALID_ARG";
        case GS_ERR_UNSUPPORTED_SIZE: return "GS_ERR_UNSUPPORTED_SIZE";
        case GS_ERR_ACCURACY: return "GS_ERR_ACCURACY";
        case GS_ERR_OUT_OF_MEMORY: return "GS_ERR_OUT_OF_MEMORY";
        case GS_ERR_NO_DEVICE: return "GS_ERR_NO_DEVICE";
        case GS_ERR_HIP: return "GS_ERR_HIP";
    }
    return "GS_UNKNOWN_STATUS";
}

const char* gs_last_error(void) { return g_err.c_str(); }

int gs_device_count(void) { return visible_devices(); }

int gs_supported_sizes(int d, int64_t* out, int capacity) {
    if (d != 2 && d != 3) return 0;
    std::vector<long long> tmp(64);
    const int c = gsk::eval_sizes(d, tmp.data(), 64);
    for (int i = 0; i < c && i < capacity && out; ++i) out[i] = tmp[i];
    return c;
}

gs_status gs_plan_create(gs_plan* out, gs_kernel k, int d, const int64_t* n, const double* L, double eps,
                         const gs_options* opt_in) {
    if (!out) return fail(GS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    gs_options opt;
    gs_options_default(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.delta_rel == 0.0) opt.delta_rel = 1e-4;
    if (d != 2 && d != 3) return fail(GS_ERR_INVALID_ARG, "d must be 2 or 3");
    if (!n || !L) return fail(GS_ERR_INVALID_ARG, "n or L is NULL");
    const int want_d = (k == GS_COULOMB_3D || k == GS_DIPOLAR_3D) ? 3
                     : (k == GS_COULOMB_2D || k == GS_POISSON_2D || k == GS_DAVEY_STEWARTSON_2D) ? 2 : d;
    if (k < GS_COULOMB_3D || k > GS_INVERSE_POWER) return fail(GS_ERR_INVALID_ARG, "unknown kernel");
    if (k == GS_INVERSE_POWER && !(opt.beta > 0.0 && opt.beta < d))
        return fail(GS_ERR_INVALID_ARG, "inverse power: beta must lie in (0, d)");
    if (want_d != d) return fail(GS_ERR_INVALID_ARG, "kernel and dimension disagree");
    double Lmax = 0.0, Lmin = 0.0, sum2 = 0.0;
    for (int i = 0; i < d; ++i) {
        if (n[i] < 2 || n[i] > 1 << 20) return fail(GS_ERR_INVALID_ARG, "n out of range");
        if (!(L[i] > 0.0) || !std::isfinite(L[i])) return fail(GS_ERR_INVALID_ARG, "L must be positive");
        Lmax = std::max(Lmax, L[i]);
        Lmin = (i == 0) ? L[i] : std::min(Lmin, L[i]);
    }
    for (int i = 0; i < d; ++i) sum2 += (L[i] / Lmax) * (L[i] / Lmax);
    // the near-field ball of the Taylor correction must fit the shortest axis
    if (k != GS_GAUSSIAN_SUM && !(opt.delta_rel < Lmin / Lmax))
        return fail(GS_ERR_INVALID_ARG, "delta_rel must be below the shortest half-width over the largest");
    if (!(opt.delta_rel > 0.0 && opt.delta_rel < 0.5)) return fail(GS_ERR_INVALID_ARG, "delta_rel out of (0, 0.5)");
    if (k != GS_GAUSSIAN_SUM && !(eps > 0.0 && eps < 1.0)) return fail(GS_ERR_INVALID_ARG, "eps out of (0, 1)");
    if (k != GS_GAUSSIAN_SUM && eps < 1e-15)
        return fail(GS_ERR_ACCURACY, "eps below the double-precision floor of the Gaussian-sum tables");
    // padding 3 (B_3): the transforms of length 3 n_j run as the padding 2 of a grid of
    // 3 n_j / 2 points (the density in its first n_j points, zeros after), which needs n_j even
    const int pad = (opt.flags & GS_PLAN_PAD3) ? 3 : 2;
    int nc[3] = {1, 1, 1}, nk[3] = {1, 1, 1}, nu[3] = {1, 1, 1};
    bool cube = true;
    for (int i = 0; i < d; ++i) {
        nc[i] = (int)n[i];
        nu[i] = (int)n[d - 1 - i];
        if (pad == 3 && nu[i] % 2 != 0)
            return fail(GS_ERR_INVALID_ARG, "padding to B_3 needs an even number of points on every axis");
        nk[i] = pad == 3 ? 3 * nu[i] / 2 : nu[i];
        cube = cube && n[i] == n[0];
        if (!gsk::eval_size_supported(d, nk[i]))
            return fail(GS_ERR_UNSUPPORTED_SIZE, "no kernels compiled for transforms of n = " + std::to_string(nk[i]) +
                                                     (pad == 3 ? " (3/2 of the grid's points)" : ""));
    }
    const int nn = *std::max_element(nc, nc + d);
    const bool host_only = (opt.flags & GS_PLAN_HOST_ONLY) != 0;
    const bool no_ws = (opt.flags & GS_PLAN_NO_WORKSPACE) != 0;
    if ((opt.flags & GS_PLAN_UNPADDED_LAPLACIAN) && (k == GS_DIPOLAR_3D || k == GS_DAVEY_STEWARTSON_2D))
        return fail(GS_ERR_INVALID_ARG, "the unpadded-grid Laplacian applies to kernels whose Taylor term acts on "
                                        "rho itself (not the dipolar or Davey-Stewartson source)");
    if (no_ws && (opt.flags & GS_PLAN_AUTOTUNE))
        return fail(GS_ERR_INVALID_ARG, "GS_PLAN_AUTOTUNE times gs_eval, which needs the workspace "
                                        "GS_PLAN_NO_WORKSPACE leaves out");
    if (k == GS_GAUSSIAN_SUM) {
        if (!opt.gs_w || !opt.gs_tau || opt.gs_q <= 0) return fail(GS_ERR_INVALID_ARG, "custom Gaussian sum missing");
        for (int q = 0; q < opt.gs_q; ++q)
            if (!(opt.gs_tau[q] >= 0.0) || !std::isfinite(opt.gs_w[q]))
                return fail(GS_ERR_INVALID_ARG, "custom Gaussian sum: tau must be >= 0, w finite");
    }
    if (k == GS_DIPOLAR_3D) {
        // The dipolar operator is bilinear in (n, m); vectors are used as given
        // (printed orientations are unit only to their printed digits).
        double a = 0, b = 0;
        for (int i = 0; i < 3; ++i) {
            a += opt.dipole_n[i] * opt.dipole_n[i];
            b += opt.dipole_m[i] * opt.dipole_m[i];
        }
        if (!std::isfinite(a) || !std::isfinite(b) || a == 0.0 || b == 0.0)
            return fail(GS_ERR_INVALID_ARG, "dipole vectors must be finite and non-zero");
    }
    {
        const size_t nx = nk[0], ny = nk[1], nz = d == 3 ? nk[2] : 1;
        const size_t ws = no_ws ? 0 : (d == 3 ? 3 * (nx + 1) * ny * nz * 16 : (nx + 1) * ny * 16) +
                                          (pad == 3 ? nx * ny * nz * 8 : 0);
        const size_t spec = (nx + 1) * (ny + 1) * (d == 3 ? nz + 1 : 1) * 8;
        const size_t bytes = spec + ws + 2 * (nx + ny + nz) * 16;
        if (!host_only && bytes > workspace_cap())
            return fail(GS_ERR_OUT_OF_MEMORY, "plan exceeds GS_MAX_WORKSPACE_BYTES");
    }
    int ndev = 0;
    if (!host_only) {
        ndev = visible_devices();
        if (ndev <= 0) return fail(GS_ERR_NO_DEVICE, "no HIP device visible");
        if (opt.device >= ndev) return fail(GS_ERR_INVALID_ARG, "device ordinal out of range");
    }

    auto* p = new gs_plan_s();
    p->kernel = k;
    p->d = d;
    p->n = nn;
    p->nf = *std::max_element(nk, nk + d);
    p->pad = pad;
    p->cube = cube;
    for (int i = 0; i < 3; ++i) {
        p->nc[i] = nc[i];
        p->nk[i] = nk[i];
        p->nu[i] = nu[i];
    }
    p->L = Lmax;
    for (int i = 0; i < d; ++i) {
        p->Lc[i] = L[i];
        // octant axes x, y[, z]: C order reversed; with padding 3 the transform grid has the
        // same step on 3/2 the half-width (its padded box is B_3)
        p->Lk[i] = pad == 3 ? 1.5 * L[d - 1 - i] : L[d - 1 - i];
    }
    p->eps = eps;
    p->delta_rel = opt.delta_rel;
    p->flags = opt.flags;
    p->host_only = host_only;
    p->tile_bits = opt.tile_variants & 8191;
    if (opt.launch_hints > 0) p->hint_bits = (opt.launch_hints - 1) & 31;
    p->stream = (hipStream_t)opt.stream;
    for (int i = 0; i < 3; ++i) {
        p->dn[i] = opt.dipole_n[i];
        p->dm[i] = opt.dipole_m[i];
    }

    bool ok = true;
    const double hi = 2.0 * std::sqrt(sum2);   // largest distance in the box, in units of L
    if (k == GS_COULOMB_3D || k == GS_DIPOLAR_3D || k == GS_COULOMB_2D) {
        ok = gsh::coulomb_table(d, p->L, hi, p->delta_rel, eps, p->table);
    } else if (k == GS_POISSON_2D || k == GS_DAVEY_STEWARTSON_2D) {
        ok = gsh::poisson_table(p->L, hi, p->delta_rel, eps, p->table);
    } else if (k == GS_INVERSE_POWER) {
        ok = gsh::power_table(opt.beta, p->L, hi, p->delta_rel, eps, p->table);
    } else {
        p->table.w.assign(opt.gs_w, opt.gs_w + opt.gs_q);
        p->table.tau.assign(opt.gs_tau, opt.gs_tau + opt.gs_q);
        p->table.S = opt.gs_q - 1;
        p->table.delta = 0.0;
    }
    if (!ok) {
        delete p;
        return fail(GS_ERR_ACCURACY, "eps not reachable by the sinc Gaussian sum");
    }
    for (int i = 0; i < d; ++i) {
        int same = -1;
        for (int j = 0; j < i; ++j)
            if (p->Lk[j] == p->Lk[i] && p->nk[j] == p->nk[i]) same = j;
        // integrals over [-2 L_j, 2 L_j] (eq. (tensor)) at the padded grid's frequencies
        if (same >= 0) p->Fk[i] = p->Fk[same];
        else gsh::factors_1d(p->table.tau, L[d - 1 - i], p->nk[i], p->Fk[i], pad);
    }
    gsh::taylor_constants(k, d, p->table, p->A0, p->c2);

    const size_t n1 = (size_t)nk[0] + 1;       // kx planes
    p->spec_bytes = n1 * (nk[1] + 1) * (d == 3 ? nk[2] + 1 : 1) * sizeof(double);
    const size_t x1 = n1 * nk[1] * (d == 3 ? (size_t)nk[2] : 1);
    size_t x2 = 0;
    if (d == 3) {
        // kx slab of the middle passes; X2 (2 ny nz complex per plane) holds one slab, or
        // every plane when slab chains run concurrently
        const size_t plane = 2 * (size_t)nk[1] * nk[2] * sizeof(double2);
        int per = (int)n1;
        if (opt.slab_planes > 0) per = std::min<int>(opt.slab_planes, (int)n1);
        else if (opt.slab_planes == 0) per = (int)std::max<size_t>(1, std::min<size_t>(n1, slab_budget() / plane));
        const int nsl = (int)((n1 + per - 1) / per);
        const int slab = (int)((n1 + nsl - 1) / nsl);
        p->x2_planes = opt.slab_streams > 1 ? (int)n1 : slab;
        (void)set_slabs(p, slab, std::max(1, opt.slab_streams));
        x2 = plane / sizeof(double2) * (size_t)p->x2_planes;
    } else {
        p->slab = (int)n1;
        p->steps = {{1, 0}, {3, 0}, {5, 0}};
    }
    // twiddle tables: one of length n for a cube, else one per distinct axis length
    size_t tw_bytes = 0;
    for (int i = 0; i < d; ++i) {
        bool seen = false;
        for (int j = 0; j < i; ++j) seen = seen || nk[j] == nk[i];
        if (!seen) tw_bytes += 2 * (size_t)nk[i] * sizeof(double2);
    }
    const size_t ebytes = pad == 3 ? (size_t)nk[0] * nk[1] * (d == 3 ? nk[2] : 1) * sizeof(double) : 0;
    p->work_bytes = (no_ws ? 0 : (x1 + x2) * sizeof(double2) + ebytes) + tw_bytes;
    const int lapu = (opt.flags & GS_PLAN_UNPADDED_LAPLACIAN) ? pad : 0;

    if (host_only) {
        gsh::assemble_spectrum(d, p->nk, p->Lk, p->table, p->Fk, p->A0, p->c2, k == GS_DAVEY_STEWARTSON_2D, lapu,
                               p->spec_host);
        log(1, "host-only plan kernel=%d d=%d n=(%d, %d, %d) L=(%g, %g, %g) S=%d Q=%zu delta=%.3g A0=%.6g c2=%.6g",
            (int)k, d, p->nc[0], p->nc[1], p->nc[2], p->Lc[0], p->Lc[1], p->Lc[2], p->table.S, p->table.w.size(),
            p->table.delta, p->A0, p->c2);
        std::lock_guard<std::mutex> g(g_live_mu);
        g_live.insert(p);
        *out = p;
        return GS_OK;
    }

    if (opt.device < 0) {
        if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
    } else {
        p->device = opt.device;
    }
    gs_status st = GS_OK;
    {
        DeviceScope ds(p->device);
        hipError_t e = ds.err;
        if (e != hipSuccess) st = hip_fail(e, "hipSetDevice");
        if (st == GS_OK && (e = hipMalloc(&p->spec, p->spec_bytes)) != hipSuccess)
            st = fail(GS_ERR_OUT_OF_MEMORY, "hipMalloc(spectrum) failed");
        if (st == GS_OK && !no_ws && (e = hipMalloc(&p->X1, x1 * sizeof(double2))) != hipSuccess)
            st = fail(GS_ERR_OUT_OF_MEMORY, "hipMalloc(workspace X1) failed");
        if (st == GS_OK && !no_ws && x2 && (e = hipMalloc(&p->X2, x2 * sizeof(double2))) != hipSuccess)
            st = fail(GS_ERR_OUT_OF_MEMORY, "hipMalloc(workspace X2) failed");
        if (st == GS_OK && !no_ws && ebytes && (e = hipMalloc(&p->E, ebytes)) != hipSuccess)
            st = fail(GS_ERR_OUT_OF_MEMORY, "hipMalloc(workspace E) failed");
        // per-axis twiddle tables (the cubic passes use tw, which is the x axis' table)
        for (int i = 0; i < d && st == GS_OK; ++i) {
            int same = -1;
            for (int j = 0; j < i; ++j)
                if (nk[j] == nk[i]) same = j;
            if (same >= 0) {
                p->twk[i] = p->twk[same];
                continue;
            }
            if ((e = hipMalloc(&p->twk[i], 2 * (size_t)nk[i] * sizeof(double2))) != hipSuccess) {
                st = fail(GS_ERR_OUT_OF_MEMORY, "hipMalloc(twiddles) failed");
                break;
            }
            std::vector<double> tw;
            gsh::twiddles(nk[i], tw);
            if ((e = hipMemcpy(p->twk[i], tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
                st = hip_fail(e, "hipMemcpy(twiddles)");
        }
        if (st == GS_OK) p->tw = p->twk[0];
        if (st == GS_OK && !no_ws &&
            (e = hipMalloc(&p->epart, ((size_t)gsk::energy_pencils(d, nk[0], nk[1]) + gsk::energy_total_scratch()) *
                                          sizeof(double))) !=
                hipSuccess)
            st = fail(GS_ERR_OUT_OF_MEMORY, "hipMalloc(energy partial sums) failed");
        if (st == GS_OK && (e = hipMalloc(&p->mixpart, mixture_partial_doubles() * sizeof(double))) != hipSuccess)
            st = fail(GS_ERR_OUT_OF_MEMORY, "hipMalloc(mixture partial sums) failed");
        if (st == GS_OK) {
            if (opt.flags & GS_PLAN_HOST_ASSEMBLY) {
                gsh::assemble_spectrum(d, p->nk, p->Lk, p->table, p->Fk, p->A0, p->c2, k == GS_DAVEY_STEWARTSON_2D,
                                       lapu, p->spec_host);
                if ((e = hipMemcpy(p->spec, p->spec_host.data(), p->spec_bytes, hipMemcpyHostToDevice)) != hipSuccess)
                    st = hip_fail(e, "hipMemcpy(spectrum)");
            } else {
                st = device_assembly(p);
            }
        }
    }
    if (st != GS_OK) {
        free_device(p);
        delete p;
        (void)hipGetLastError();
        return st;
    }
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        g_live.insert(p);
    }
    log(1, "plan kernel=%d d=%d n=%d L=(%g, %g, %g) S=%d Q=%zu delta=%.3g A0=%.6g c2=%.6g spectrum %zu B, "
        "workspace %zu B, assembly %.3f ms", (int)k, d, nn, p->Lc[0], p->Lc[1], p->Lc[2], p->table.S,
        p->table.w.size(), p->table.delta, p->A0, p->c2, p->spec_bytes, p->work_bytes, p->assembly_ms);
    if (opt.flags & GS_PLAN_AUTOTUNE) {
        // the plan is complete: the autotuner times it through the ordinary eval path
        st = plan_autotune(p);
        if (st != GS_OK) {
            (void)gs_plan_destroy(p);
            (void)hipGetLastError();
            return st;
        }
    }
    *out = p;
    return GS_OK;
}

gs_status gs_plan_destroy(gs_plan p) {
    if (!p) return GS_OK;
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        if (!g_live.count(p)) return GS_OK;          // already destroyed: no-op
        g_live.erase(p);
    }
    free_device(p);
    delete p;
    return GS_OK;
}

gs_status gs_plan_query(gs_plan p, gs_plan_info* info) {
    if (!is_live(p) || !info) return fail(GS_ERR_INVALID_ARG, "invalid plan or info");
    std::memset(info, 0, sizeof(*info));
    info->kernel = p->kernel;
    info->d = p->d;
    info->n = p->n;
    info->L = p->L;
    for (int i = 0; i < p->d; ++i) {
        info->L_axes[i] = p->Lc[i];
        info->n_axes[i] = p->nc[i];
    }
    info->padding = p->pad;
    info->beta = p->table.beta;
    info->eps = p->eps;
    info->delta = p->table.delta;
    info->S = p->table.S;
    info->Q = (int)p->table.w.size();
    info->A0 = p->A0;
    info->c2 = p->c2;
    info->spectrum_bytes = p->spec_bytes;
    info->workspace_bytes = p->work_bytes;
    info->assembly_ms = p->assembly_ms;
    info->assembly_gflop = 2.0 * info->Q * (p->nk[0] + 1.0) * (p->nk[1] + 1.0) * (p->d == 3 ? p->nk[2] + 1.0 : 1.0) * 1e-9;
    info->host_only = p->host_only ? 1 : 0;
    info->slab_planes = p->slab;
    info->num_steps = (int)p->steps.size();
    info->slab_streams = p->nstreams;
    info->x2_planes = p->d == 3 ? p->x2_planes : 0;
    info->tuned = p->tuned ? 1 : 0;
    info->hint_bits = p->hint_bits;
    info->fused_grid_mult = p->fused_mult;
    info->tile_variants = p->tile_bits;
    info->tune_candidates = p->tune_candidates;
    info->tuned_ms = p->tuned_ms;
    return GS_OK;
}

gs_status gs_plan_table(gs_plan p, double* w, double* tau, int capacity) {
    if (!is_live(p) || !w || !tau) return fail(GS_ERR_INVALID_ARG, "invalid plan or pointer");
    const int Q = (int)p->table.w.size();
    if (capacity < Q) return fail(GS_ERR_INVALID_ARG, "capacity too small");
    std::memcpy(w, p->table.w.data(), Q * sizeof(double));
    std::memcpy(tau, p->table.tau.data(), Q * sizeof(double));
    return GS_OK;
}

gs_status gs_plan_factors_axis(gs_plan p, int axis, double* F, size_t capacity) {
    if (!is_live(p) || !F) return fail(GS_ERR_INVALID_ARG, "invalid plan or pointer");
    if (axis < 0 || axis >= p->d) return fail(GS_ERR_INVALID_ARG, "axis out of range");
    const std::vector<double>& Fa = p->Fk[p->d - 1 - axis];
    if (capacity < Fa.size()) return fail(GS_ERR_INVALID_ARG, "capacity too small");
    std::memcpy(F, Fa.data(), Fa.size() * sizeof(double));
    return GS_OK;
}

gs_status gs_plan_factors(gs_plan p, double* F, size_t capacity) {
    if (!is_live(p)) return fail(GS_ERR_INVALID_ARG, "invalid plan or pointer");
    return gs_plan_factors_axis(p, p->d - 1, F, capacity);
}

gs_status gs_plan_spectrum(gs_plan p, double* host_out, size_t capacity) {
    if (!is_live(p) || !host_out) return fail(GS_ERR_INVALID_ARG, "invalid plan or pointer");
    const size_t cnt = p->spec_bytes / sizeof(double);
    if (capacity < cnt) return fail(GS_ERR_INVALID_ARG, "capacity too small");
    if (p->host_only) {
        std::memcpy(host_out, p->spec_host.data(), p->spec_bytes);
        return GS_OK;
    }
    DeviceScope ds(p->device);
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess) e = hipMemcpy(host_out, p->spec, p->spec_bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(spectrum)");
    return GS_OK;
}

gs_status gs_plan_buffer(gs_plan p, int which, int to_device, double* host, size_t count) {
    if (!is_live(p) || !host) return fail(GS_ERR_INVALID_ARG, "invalid plan or pointer");
    if (p->host_only) return fail(GS_ERR_INVALID_ARG, "host-only plan has no device buffers");
    const size_t nx = p->nk[0], ny = p->nk[1], nz = p->d == 3 ? p->nk[2] : 1;
    void* buf = nullptr;
    size_t doubles = 0;
    if ((which == 1 || which == 2) && !p->X1) return fail(GS_ERR_INVALID_ARG, "plan has no workspace");
    if (which == 1) {
        buf = p->X1;
        doubles = 2 * (nx + 1) * ny * nz;
    } else if (which == 2 && p->d == 3) {
        buf = p->X2;
        doubles = 2 * 2 * ny * nz * (size_t)p->x2_planes;
    } else if (which == 3) {
        buf = p->spec;
        doubles = p->spec_bytes / sizeof(double);
    } else {
        return fail(GS_ERR_INVALID_ARG, "unknown buffer");
    }
    if (count != doubles) return fail(GS_ERR_INVALID_ARG, "count does not match the buffer size");
    DeviceScope ds(p->device);
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess)
        e = to_device ? hipMemcpy(buf, host, count * sizeof(double), hipMemcpyHostToDevice)
                      : hipMemcpy(host, buf, count * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(plan buffer)");
    return GS_OK;
}

gs_status gs_plan_set_stream(gs_plan p, void* stream) {
    if (!is_live(p)) return fail(GS_ERR_INVALID_ARG, "invalid plan");
    p->stream = (hipStream_t)stream;
    return GS_OK;
}

gs_status gs_eval(gs_plan p, const double* rho_dev, double* u_dev) { return eval_chain(p, rho_dev, u_dev, -1); }

gs_status gs_eval_energy(gs_plan p, const double* rho_dev, double* u_dev, double* energy_dev) {
    if (!energy_dev) return fail(GS_ERR_INVALID_ARG, "NULL energy pointer");
    return eval_chain(p, rho_dev, u_dev, -1, energy_dev);
}

gs_status gs_eval_energy_gradient(gs_plan p, const double* rho_dev, double* grad_dev, double* energy_dev) {
    if (!energy_dev) return fail(GS_ERR_INVALID_ARG, "NULL energy pointer");
    return eval_chain(p, rho_dev, grad_dev, -1, energy_dev, true);
}

gs_status gs_eval_backward(gs_plan p, const double* grad_u_dev, double* grad_rho_dev) {
    // The transposed chain: zero-pad <-> crop exchanged and the transform signs
    // flipped.  With an even spectrum (every supported kernel) the sign flip is
    // the index reversal k -> -k, under which the spectrum is invariant, so the
    // transposed chain is the same sequence of passes.
    return eval_chain(p, grad_u_dev, grad_rho_dev, -1);
}

gs_status gs_eval_events(gs_plan p, const double* rho_dev, double* u_dev, void* const* events, int count) {
    if (!is_live(p)) return fail(GS_ERR_INVALID_ARG, "invalid plan");
    if (!events || count != (int)p->steps.size() + 1) return fail(GS_ERR_INVALID_ARG, "need one event per step plus one");
    gsk::EvalArgs a;
    gs_status st = make_args(p, rho_dev, u_dev, a);
    if (st != GS_OK) return st;
    if (!p->X1) return fail(GS_ERR_INVALID_ARG, "plan created without a workspace (GS_PLAN_NO_WORKSPACE)");
    DeviceScope ds(p->device);
    if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
    // a NULL handle records nothing (each record costs the stream a few microseconds)
    hipError_t e = events[0] ? hipEventRecord((hipEvent_t)events[0], p->stream) : hipSuccess;
    for (int i = 0; i < (int)p->steps.size() && e == hipSuccess; ++i) {
        e = run_step(p, a, i, p->stream);
        if (e == hipSuccess && events[i + 1]) e = hipEventRecord((hipEvent_t)events[i + 1], p->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "evaluation launch");
    return GS_OK;
}

gs_status gs_eval_step(gs_plan p, const double* rho_dev, double* u_dev, int step) {
    if (step < 0) return fail(GS_ERR_INVALID_ARG, "step must be >= 0");
    return eval_chain(p, rho_dev, u_dev, step);
}

int gs_plan_steps(gs_plan p, int* pass_ids, int capacity) {
    if (!is_live(p)) return -1;
    const int c = (int)p->steps.size();
    for (int i = 0; i < c && i < capacity && pass_ids; ++i) pass_ids[i] = p->steps[i].first;
    return c;
}

}  // extern "C"

namespace {

// Times whole evaluations of p (launch variants in p) on scratch buffers: best of 3
// after one warm-up, in ms.
gs_status time_plan(gs_plan_s* p, const double* rho, double* u, double& ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    gs_status st = eval_chain(p, rho, u, -1);
    ms = 1e300;
    for (int r = 0; r < 3 && st == GS_OK; ++r) {
        (void)hipEventRecord(e0, p->stream);
        st = eval_chain(p, rho, u, -1);
        (void)hipEventRecord(e1, p->stream);
        const hipError_t e = hipEventSynchronize(e1);
        if (e != hipSuccess) st = hip_fail(e, "autotune timing");
        float f = 0.f;
        (void)hipEventElapsedTime(&f, e0, e1);
        ms = std::min(ms, (double)f);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

// Greedy search over the launch variants: starting from the compiled defaults, flip each
// pass's cache-hint variant in turn and keep what is faster, then try one and four rounds of
// co-resident blocks in the fused pass, then the tile shapes and the radix plans.  None but
// the radix plans changes the result (they agree with the default to rounding).  Timed on
// scratch buffers, so the caller's data is never evaluated by a candidate.
gs_status plan_autotune(gs_plan_s* p) {
    std::string dims = std::to_string(p->nc[0]);
    for (int i = 1; i < p->d; ++i) dims += "x" + std::to_string(p->nc[i]);
    const std::string key = tune_device_key(p->device) + "|plan|d" + std::to_string(p->d) + "|n" + dims +
                            (p->kernel == GS_DIPOLAR_3D ? "|dip" : "") + (p->pad == 3 ? "|pad3" : "") + "|slab" +
                            std::to_string(p->slab);
    TuneEntry te;
    if (tune_lookup(key, te)) {
        p->hint_bits = te.schedule;
        p->fused_mult = te.tiles_per_task;
        p->tile_bits = te.grid;
        p->tuned = true;
        p->tuned_ms = te.ms;
        return GS_OK;
    }
    const size_t pts = (size_t)p->nc[0] * p->nc[1] * (p->d == 3 ? p->nc[2] : 1);
    double *rho = nullptr, *u = nullptr;
    if (hipMalloc(&rho, pts * sizeof(double)) != hipSuccess || hipMalloc(&u, pts * sizeof(double)) != hipSuccess) {
        if (rho) (void)hipFree(rho);
        (void)hipGetLastError();
        return fail(GS_ERR_OUT_OF_MEMORY, "autotune scratch allocation failed");
    }
    gs_status st = GS_OK;
    hipError_t e = hipMemsetAsync(rho, 0, pts * sizeof(double), p->stream);
    if (e != hipSuccess) st = hip_fail(e, "autotune scratch");
    double best = 1e300;
    if (st == GS_OK) st = time_plan(p, rho, u, best);
    const int passes[5] = {1, 2, 3, 4, 5};
    for (int pass : passes) {
        if (st != GS_OK) break;
        if (p->d == 2 && (pass == 2 || pass == 4)) continue;
        const int keep = p->hint_bits;
        p->hint_bits ^= 1 << (pass - 1);
        double ms = 0;
        st = time_plan(p, rho, u, ms);
        p->tune_candidates++;
        if (st == GS_OK && ms < best) best = ms;
        else p->hint_bits = keep;
    }
    for (int m : {1, 4}) {
        if (st != GS_OK || !p->cube || !gs_fused_persistent(p->d, p->nf)) break;   // grid fixed by the group count
        const int keep = p->fused_mult;
        p->fused_mult = m;
        double ms = 0;
        st = time_plan(p, rho, u, ms);
        p->tune_candidates++;
        if (st == GS_OK && ms < best) best = ms;
        else p->fused_mult = keep;
    }
    // tile shapes of the cubic passes: each pass type's variants in turn (x: twice the row
    // pairs; y and fused: half and twice the pencils per block), keeping what is faster; last
    // the fused pass's radix-plan variant (its own pencils per block; it rounds differently,
    // so it is kept only if faster by more than 1 %, beyond the spread of repeated timings), and
    // the x and y passes' radix-plan variants likewise
    const int tv = p->cube ? gsk::tile_variants(p->nf) : 0;
    const int tries[11][2] = {{0, 1}, {6, 1}, {2, 1}, {2, 2}, {4, 1}, {4, 2},
                              {8, 1}, {9, 1}, {10, 1}, {11, 1}, {12, 1}};   // (bit offset, value)
    const int avail[11] = {1, 1, 2, 4, 8, 16, 32, 64, 64, 128, 128};
    for (int i = 0; i < 11 && st == GS_OK; ++i) {
        const bool ypass = tries[i][0] == 2 || tries[i][0] == 11 || tries[i][0] == 12;
        if (!(tv & avail[i]) || (p->d == 2 && ypass)) continue;
        const int keep = p->tile_bits;
        const int field = tries[i][0] >= 8 ? 1 : 3;      // one-bit fields from bit 8 on
        p->tile_bits = (p->tile_bits & ~(field << tries[i][0])) | (tries[i][1] << tries[i][0]);
        double ms = 0;
        st = time_plan(p, rho, u, ms);
        p->tune_candidates++;
        const double margin = tries[i][0] >= 8 ? 0.99 : 1.0;
        if (st == GS_OK && ms < margin * best) best = ms;
        else p->tile_bits = keep;
    }
    (void)hipStreamSynchronize(p->stream);
    (void)hipFree(rho);
    (void)hipFree(u);
    if (st != GS_OK) return st;
    p->tuned = true;
    p->tuned_ms = best;
    log(1, "plan autotune n=%d d=%d: hint bits %d, fused rounds %d, tile bits %d, %.4f ms (%d variants timed)",
        p->n, p->d, p->hint_bits, p->fused_mult, p->tile_bits, best, p->tune_candidates);
    te.schedule = p->hint_bits;          // plan entries: schedule = hint bits,
    te.tiles_per_task = p->fused_mult;   // tiles_per_task = fused grid rounds,
    te.largest_first = 0;
    te.grid = p->tile_bits;              // grid = tile-shape bits
    te.ms = best;
    tune_store(key, te);
    return GS_OK;
}

}  // namespace
