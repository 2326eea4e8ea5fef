// api_internal.hpp -- the plan object and helpers shared by the C ABI sources.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/gs.h"
#include "device_api.hpp"
#include "host_plan.hpp"

struct gs_plan_s {
    int kernel = 0, d = 0, n = 0;             // n: points per axis of a cubic grid, else the largest
    int nc[3] = {0, 0, 0};                    // points per axis, C order (z, y, x / y, x)
    int nk[3] = {0, 0, 0};                    // transform points of the octant axes x, y[, z]
    int nu[3] = {0, 0, 0};                    // points of the density's grid on the octant axes
    int pad = 2;                              // zero padding to [-pad L, pad L] (2, or 3: B_3)
    int nf = 0;                               // transform points per axis (cubic), else the largest
    bool cube = true;                         // every axis has the same n
    double L = 0, eps = 0, delta_rel = 0;     // L: largest half-width (the table's length unit)
    double Lc[3] = {0, 0, 0};                 // half-widths as given, C order (z, y, x / y, x)
    double Lk[3] = {0, 0, 0};                 // half-widths of the transform grid's octant axes x, y[, z]
                                              // (pad 3: 3/2 of the density's, see gs_plan_create)
    gsh::Table table;
    std::vector<double> Fk[3];                // factors (n+1) x Q of the octant axes x, y[, z]
    double A0 = 0, c2 = 0;
    std::vector<double> spec_host;
    double dn[3] = {0, 0, 0}, dm[3] = {0, 0, 0};
    int device = 0, flags = 0;
    bool host_only = false;
    hipStream_t stream = nullptr;
    double* spec = nullptr;
    double2* X1 = nullptr;
    double2* X2 = nullptr;
    double2* tw = nullptr;                    // twiddles of length n (cubic grids)
    double2* twk[3] = {nullptr, nullptr, nullptr};   // per octant axis (rectangular grids; may alias)
    double* epart = nullptr;                  // per-pencil energy sums of the fused pass
    double* mixpart = nullptr;                // per-block sums of the mixture gradient
    double* E = nullptr;                      // pad 3: the density and potential on the transform grid
    size_t spec_bytes = 0, work_bytes = 0;
    double assembly_ms = 0.0;
    int slab = 0, nslabs = 1;                 // 3D: kx planes per slab of the middle passes
    int hint_bits = 27, fused_mult = 4;       // launch variants (see gsk::EvalArgs)
    int tile_bits = 0;                        // tile shapes of the cubic passes (gsk::EvalArgs)
    int x2_planes = 0;                        // kx planes X2 holds (n+1: every slab at its own planes)
    int nstreams = 1;                         // concurrent slab chains of the middle passes
    std::vector<hipStream_t> sstreams;        // their streams (created on demand)
    std::vector<hipEvent_t> sevents;          // one per stream, plus the fork event last
    bool tuned = false;
    int tune_candidates = 0;
    double tuned_ms = 0.0;
    std::vector<std::pair<int, int>> steps;   // (pass, slab index) in execution order
};

namespace gsapi {

// Records msg as this thread's last error and returns s.
gs_status fail(gs_status s, const std::string& msg);
// Writes one line "[gs] ..." to stderr when the environment variable GS_LOG_LEVEL is at
// least `level` (1: plan and batch decisions, 2: also every error status).
void log(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
gs_status hip_fail(hipError_t e, const char* what);
// true while p is a plan created and not yet destroyed
bool is_live(gs_plan p);

// Makes the plan's device current for the scope and restores the caller's.
struct DeviceScope {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Device arguments of one evaluation of plan p on (in, out).
gs_status make_args(gs_plan p, const double* in, double* out, gsk::EvalArgs& a);
// Queues the evaluation steps of p on its stream: all of them (step < 0) or one.  With
// energy != nullptr the last pass also forms energy[0] = 1/2 cell sum in*out.
gs_status eval_chain(gs_plan p, const double* in, double* out, int step, double* energy = nullptr,
                     bool gradient = false);
// Doubles of the per-block partial sums the mixture gradient needs (plan-owned).
size_t mixture_partial_doubles();
// Complex values of the evaluation workspace of p (X1, in 3D X2 of x2_planes planes, and
// with padding 3 the transform-grid copy E of the density).
size_t workspace_complex(gs_plan p);
// Queues every evaluation step of p on its stream with its workspace in ws (device memory
// of workspace_complex(p) complex values: X1, then X2, then E), in order.
gs_status eval_chain_ws(gs_plan p, const double* in, double* out, double2* ws);
// Rebuilds p's step list for `planes` kx planes per slab (3D), run on `streams` streams
// (X2 must hold every plane when streams > 1 or planes exceed x2_planes: returns false).
bool set_slabs(gs_plan p, int planes, int streams);

}  // namespace gsapi
