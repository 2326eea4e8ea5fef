// static_eval.hip -- gs_eval_static: the evaluation with its workspace in a fixed device
// array instead of the plan's own (include/gs.h), for callers that cannot allocate device
// memory when they evaluate (code under stream capture, tight serving loops).
//
// The workspace of an evaluation (X1 and, in 3D, X2: the intermediate transforms between
// the passes) lives in `scratch`, a file-scope device array of GS_STATIC_SCRATCH_BYTES.
// Every device the library runs on holds its own copy from the time the library's code is
// loaded there until the process ends.  Host code never passes the array's name to a
// kernel (on the host that name is a stand-in, not a device address): on the first call
// on a device, with that device current, hipGetSymbolAddress gives that device's address,
// which is kept per device and used for every launch.
//
// The passes write every workspace element before reading it, so nothing needs clearing
// between calls.  Calls on one device share the array: calls that overlap in time on one
// device (concurrent streams, several threads) race and must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/gs.h"
#include "api_internal.hpp"

namespace {

constexpr size_t kScratchComplex = GS_STATIC_SCRATCH_BYTES / sizeof(double2);
static_assert(GS_STATIC_SCRATCH_BYTES % 256 == 0, "whole 256-byte lines");

static __device__ __align__(256) double2 scratch[kScratchComplex];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double2* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev` (looked up once per device, that device current).
gs_status scratch_on(int dev, double2*& out) {
    if (dev < 0 || dev >= kMaxDevices) return gsapi::fail(GS_ERR_INVALID_ARG, "device ordinal out of range");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        gsapi::DeviceScope ds(dev);
        if (ds.err != hipSuccess) return gsapi::hip_fail(ds.err, "hipSetDevice");
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return gsapi::hip_fail(e, "hipGetSymbolAddress(static scratch)");
        g_scratch_ptr[dev] = static_cast<double2*>(ptr);
    }
    out = g_scratch_ptr[dev];
    return GS_OK;
}

}  // namespace

extern "C" gs_status gs_eval_static(gs_plan p, const double* rho_dev, double* u_dev) {
    if (!gsapi::is_live(p)) return gsapi::fail(GS_ERR_INVALID_ARG, "invalid plan");
    if (p->host_only) return gsapi::fail(GS_ERR_INVALID_ARG, "host-only plan cannot evaluate");
    if (!rho_dev || !u_dev) return gsapi::fail(GS_ERR_INVALID_ARG, "NULL device pointer");
    const size_t need = gsapi::workspace_complex(p);
    if (need > kScratchComplex)
        return gsapi::fail(GS_ERR_UNSUPPORTED_SIZE,
                           "workspace of " + std::to_string(need * sizeof(double2)) +
                               " bytes exceeds the static scratch of " + std::to_string(GS_STATIC_SCRATCH_BYTES) +
                               " bytes (it holds 3D grids up to n = 128 with the default slab, 2D grids up to n = 2048)");
    double2* ws = nullptr;
    const gs_status st = scratch_on(p->device, ws);
    if (st != GS_OK) return st;
    return gsapi::eval_chain_ws(p, rho_dev, u_dev, ws);
}
