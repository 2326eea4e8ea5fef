// mixture.hip -- Gaussian-mixture densities on a plan's grid and the parameter gradient of
// a scalar through them (include/gs.h: gs_mixture_density, gs_mixture_gradient).
//
// The density rho(x) = sum_c a_c exp(-|x - mu_c|^2 / sigma_c^2) is the input family of the
// differentiation workload; the energy's gradient with respect to the parameters is the chain
// rule from its grid gradient g = dE/drho:
//   dE/da_c        = sum_i g_i e_ci
//   dE/dmu_cj      = (2 a_c / sigma_c^2) sum_i g_i e_ci (x_ij - mu_cj)
//   dE/dsigma_c    = (2 a_c / sigma_c^3) sum_i g_i e_ci |x_i - mu_c|^2,
// e_ci = exp(-|x_i - mu_c|^2 / sigma_c^2).  Each Gaussian is a product of one-dimensional
// factors, so a block forms the (y, z) factors of its rows once (LDS) and each thread the x
// factors of its columns once per tile.  The sums are reduced in a fixed order (per thread,
// then per block by a butterfly and the waves in order, then over the blocks by one more
// launch), so the gradient is the same bits on every run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "api_internal.hpp"

namespace {

constexpr int MT = 256;          // threads per block
constexpr int ROWS = 16;         // grid rows (fixed z, y; x varying) per tile, at most
constexpr int CH = 8;            // components per gradient launch
constexpr int NS = 5;            // sums per component: S, Sx, Sy, Sz, R
constexpr int MAX_K = 64;
constexpr int GRAD_GRID = 1024;  // blocks of the gradient launch (they loop over tiles)

struct MixGeom {
    int d, n, ny, rows, rpt;     // points along x (a row), along y, grid rows, rows per tile
    double x0[3], h[3];          // axis x, y, z: coordinate of index i = x0 + i h
};

// Row r of the grid: (y, z) indices (2D: z = 0).
__device__ __forceinline__ void row_yz(const MixGeom& g, int r, int& y, int& z) {
    y = r % g.ny;
    z = r / g.ny;
}

// Sum of one value per thread of a 256-thread block in a fixed order; valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void __launch_bounds__(MT) k_mix_density(MixGeom g, int K, const double* __restrict__ a,
                                                    const double* __restrict__ mu, const double* __restrict__ sig,
                                                    double* __restrict__ rho) {
    __shared__ double eyz[ROWS * MAX_K];        // a_c exp(-((y - mu_y)^2 + (z - mu_z)^2) / sigma^2)
    const int r0 = blockIdx.x * g.rpt;
    for (int t = threadIdx.x; t < g.rpt * K; t += MT) {
        const int r = t / K, c = t % K;
        double v = 0.0;
        if (r0 + r < g.rows) {
            int y, z;
            row_yz(g, r0 + r, y, z);
            const double dy = g.x0[1] + y * g.h[1] - mu[c * g.d + 1];
            const double dz = g.d == 3 ? g.x0[2] + z * g.h[2] - mu[c * g.d + 2] : 0.0;
            v = a[c] * exp(-(dy * dy + dz * dz) / (sig[c] * sig[c]));
        }
        eyz[r * K + c] = v;
    }
    __syncthreads();
    for (int x = threadIdx.x; x < g.n; x += MT) {
        double acc[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) acc[r] = 0.0;
        const double px = g.x0[0] + x * g.h[0];
        for (int c = 0; c < K; ++c) {
            const double dx = px - mu[c * g.d];
            const double ex = exp(-(dx * dx) / (sig[c] * sig[c]));
#pragma unroll
            for (int r = 0; r < ROWS; ++r) acc[r] += eyz[r * K + c] * ex;
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
            if (r < g.rpt && r0 + r < g.rows) rho[(size_t)(r0 + r) * g.n + x] = acc[r];
    }
}

// Components c0 .. c0 + kc - 1 (kc <= CH): per-block sums S, Sx, Sy, Sz, R of g_i e_ci times
// 1, (x - mu_x), (y - mu_y), (z - mu_z), |x - mu|^2, into part[block][NS * CH].
__global__ void __launch_bounds__(MT) k_mix_grad(MixGeom g, int c0, int kc, const double* __restrict__ mu,
                                                 const double* __restrict__ sig, const double* __restrict__ gr,
                                                 double* __restrict__ part) {
    __shared__ double fyz[ROWS * CH], dyv[ROWS * CH], dzv[ROWS * CH];
    __shared__ double red[4];
    double acc[NS * CH];
#pragma unroll
    for (int i = 0; i < NS * CH; ++i) acc[i] = 0.0;
    const int ntiles = (g.rows + g.rpt - 1) / g.rpt;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int r0 = tile * g.rpt;
        __syncthreads();                        // the previous tile's factors are no longer read
        for (int t = threadIdx.x; t < ROWS * CH; t += MT) {
            const int r = t / CH, cc = t % CH, c = c0 + cc;
            double f = 0.0, dy = 0.0, dz = 0.0;
            if (r < g.rpt && r0 + r < g.rows && cc < kc) {
                int y, z;
                row_yz(g, r0 + r, y, z);
                dy = g.x0[1] + y * g.h[1] - mu[c * g.d + 1];
                dz = g.d == 3 ? g.x0[2] + z * g.h[2] - mu[c * g.d + 2] : 0.0;
                f = exp(-(dy * dy + dz * dz) / (sig[c] * sig[c]));
            }
            fyz[t] = f;
            dyv[t] = dy;
            dzv[t] = dz;
        }
        __syncthreads();
        for (int x = threadIdx.x; x < g.n; x += MT) {
            const double px = g.x0[0] + x * g.h[0];
            double ex[CH], dx[CH];
#pragma unroll
            for (int cc = 0; cc < CH; ++cc) {
                const int c = c0 + (cc < kc ? cc : 0);
                dx[cc] = px - mu[c * g.d];
                ex[cc] = cc < kc ? exp(-(dx[cc] * dx[cc]) / (sig[c] * sig[c])) : 0.0;
            }
            for (int r = 0; r < g.rpt; ++r) {
                if (r0 + r >= g.rows) break;
                const double gv = gr[(size_t)(r0 + r) * g.n + x];
#pragma unroll
                for (int cc = 0; cc < CH; ++cc) {
                    const double w = gv * (fyz[r * CH + cc] * ex[cc]);
                    const double dy = dyv[r * CH + cc], dz = dzv[r * CH + cc];
                    acc[NS * cc + 0] += w;
                    acc[NS * cc + 1] += w * dx[cc];
                    acc[NS * cc + 2] += w * dy;
                    acc[NS * cc + 3] += w * dz;
                    acc[NS * cc + 4] += w * ((dx[cc] * dx[cc] + dy * dy) + dz * dz);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NS * CH; ++i) {
        const double s = block_sum256(acc[i], red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * NS * CH + i] = s;
    }
}

// One block per (component, sum): the blocks' partial sums in a fixed order, scaled into the
// derivative it belongs to.
__global__ void __launch_bounds__(MT) k_mix_grad_finish(int d, int K, int c0, int kc, int nblocks, double scale,
                                                        const double* __restrict__ a,
                                                        const double* __restrict__ sig,
                                                        const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double red[4];
    const int cc = blockIdx.x / NS, s = blockIdx.x % NS;
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += MT) v += part[(size_t)b * NS * CH + blockIdx.x];
    v = block_sum256(v, red);
    if (threadIdx.x != 0 || cc >= kc) return;
    const int c = c0 + cc;
    const double sg = sig[c];
    if (s == 0) out[c] = scale * v;                                          // d/da_c
    else if (s <= d) out[K + c * d + (s - 1)] = scale * (2.0 * a[c] / (sg * sg)) * v;      // d/dmu_c
    else if (s == 4) out[K + K * d + c] = scale * (2.0 * a[c] / (sg * sg * sg)) * v;       // d/dsigma_c
}

MixGeom geom(gs_plan p) {
    MixGeom g;
    g.d = p->d;
    g.n = p->nu[0];                                // the density's grid (not the transform grid)
    g.ny = p->nu[1];
    g.rows = p->d == 3 ? p->nu[1] * p->nu[2] : p->nu[1];
    g.rpt = std::max(1, std::min(ROWS, 4096 / g.n));
    for (int j = 0; j < 3; ++j) {
        g.x0[j] = 0.0;
        g.h[j] = 0.0;
    }
    for (int j = 0; j < p->d; ++j) {               // axis j (x, y, z) is array axis d-1-j
        const double L = p->Lc[p->d - 1 - j];
        g.x0[j] = -L;
        g.h[j] = 2.0 * L / p->nu[j];
    }
    return g;
}

gs_status check_args(gs_plan p, int K, const void* a, const void* mu, const void* sig) {
    if (!gsapi::is_live(p)) return gsapi::fail(GS_ERR_INVALID_ARG, "invalid plan");
    if (p->host_only) return gsapi::fail(GS_ERR_INVALID_ARG, "host-only plan has no device");
    if (K < 1 || K > MAX_K) return gsapi::fail(GS_ERR_INVALID_ARG, "mixture: 1 <= K <= 64 components");
    if (!a || !mu || !sig) return gsapi::fail(GS_ERR_INVALID_ARG, "NULL parameter pointer");
    return GS_OK;
}

}  // namespace

namespace gsapi {
size_t mixture_partial_doubles() { return (size_t)GRAD_GRID * NS * CH; }
}  // namespace gsapi

extern "C" {

gs_status gs_mixture_density(gs_plan p, int K, const double* a, const double* mu, const double* sigma,
                             double* rho_dev) {
    gs_status st = check_args(p, K, a, mu, sigma);
    if (st != GS_OK) return st;
    if (!rho_dev) return gsapi::fail(GS_ERR_INVALID_ARG, "NULL device pointer");
    gsapi::DeviceScope ds(p->device);
    if (ds.err != hipSuccess) return gsapi::hip_fail(ds.err, "hipSetDevice");
    const MixGeom g = geom(p);
    const int blocks = (g.rows + g.rpt - 1) / g.rpt;
    k_mix_density<<<blocks, MT, 0, p->stream>>>(g, K, a, mu, sigma, rho_dev);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return gsapi::hip_fail(e, "mixture density launch");
    return GS_OK;
}

gs_status gs_mixture_gradient(gs_plan p, int K, const double* a, const double* mu, const double* sigma,
                              const double* g_dev, double scale, double* out_dev) {
    gs_status st = check_args(p, K, a, mu, sigma);
    if (st != GS_OK) return st;
    if (!g_dev || !out_dev) return gsapi::fail(GS_ERR_INVALID_ARG, "NULL device pointer");
    if (!p->mixpart) return gsapi::fail(GS_ERR_INVALID_ARG, "plan has no mixture workspace");
    gsapi::DeviceScope ds(p->device);
    if (ds.err != hipSuccess) return gsapi::hip_fail(ds.err, "hipSetDevice");
    const MixGeom g = geom(p);
    const int ntiles = (g.rows + g.rpt - 1) / g.rpt;
    const int grid = std::min(GRAD_GRID, ntiles);
    for (int c0 = 0; c0 < K; c0 += CH) {
        const int kc = std::min(CH, K - c0);
        k_mix_grad<<<grid, MT, 0, p->stream>>>(g, c0, kc, mu, sigma, g_dev, p->mixpart);
        k_mix_grad_finish<<<NS * CH, MT, 0, p->stream>>>(g.d, K, c0, kc, grid, scale, a, sigma, p->mixpart, out_dev);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return gsapi::hip_fail(e, "mixture gradient launch");
    return GS_OK;
}

}  // extern "C"
