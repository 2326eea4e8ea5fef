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
// factors: the density kernel forms the (y, z) factors of a block's rows once (LDS) and each
// thread the x factors of its columns once per tile; the gradient contracts the grid gradient
// with the x factors on the matrix cores and applies the (y, z) factors per row (k_mix_grad).
// The sums are reduced in a fixed order (per lane, then per block, then over the blocks by one
// more launch), so the gradient is the same bits on every run.
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
constexpr int MAX_ROW = 2048;    // points along x of the largest grid (its B table)

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

// The gradient sums are a contraction with one dense factor.  With the grid gradient as a
// matrix G[row][x] (row = (y, z), x along a row) and e_ci = ex_c(x) f_c(row),
//   Y[row][3 cc + k] = sum_x G[row][x] B[x][3 cc + k],  B[x][.] = ex_c(x) (1, dx_c, dx_c^2),
// and then, per row, with dy, dz, q = dy^2 + dz^2 and f = f_c(row):
//   S += f Y0,  Sx += f Y1,  Sy += f dy Y0,  Sz += f dz Y0,  R += f q Y0 + f Y2.
// Y is formed on FP64 MFMA (v_mfma_f64_16x16x4f64), never stored: each wave takes RT tiles
// of 16 rows against the 32 columns (24 used) of B and applies the row factors to its
// accumulators.

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
constexpr int BC = 32;           // columns of B (3 CH used)
constexpr int RT = 2;            // 16-row tiles per wave and round

// B of components c0 .. c0 + kc - 1 (zero beyond them), stored by column: bt[col n + x] (x
// consecutive, so a lane's four x values are one 32-byte run).  One thread per entry.
__global__ void __launch_bounds__(MT) k_mix_table(MixGeom g, int c0, int kc, const double* __restrict__ mu,
                                                  const double* __restrict__ sig, double* __restrict__ bt) {
    const int idx = blockIdx.x * MT + threadIdx.x;
    if (idx >= g.n * BC) return;
    const int col = idx / g.n, x = idx % g.n, cc = col / 3, k = col % 3;
    double v = 0.0;
    if (cc < kc) {
        const int c = c0 + cc;
        const double dx = g.x0[0] + x * g.h[0] - mu[c * g.d];
        const double ex = exp(-(dx * dx) / (sig[c] * sig[c]));
        v = k == 0 ? ex : (k == 1 ? ex * dx : ex * dx * dx);
    }
    bt[idx] = v;
}

// Four consecutive doubles p[0..3] as two 16-byte loads (every row length is a multiple of 4,
// so a lane's four values lie in one row), or those below `lim` of them with zeros after.
__device__ __forceinline__ void load4(const double* p, int lim, double (&v)[4]) {
    if (lim >= 4) {
        const v2d a = *reinterpret_cast<const v2d*>(p), b = *reinterpret_cast<const v2d*>(p + 2);
        v[0] = a.x;
        v[1] = a.y;
        v[2] = b.x;
        v[3] = b.y;
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = s < lim ? p[s] : 0.0;
    }
}

// Components c0 .. c0 + kc - 1 (kc <= CH): per-block sums S, Sx, Sy, Sz, R into
// part[block][NS * CH] (NS * cc + s), each in a fixed order (the waves' tiles in turn, the
// lanes of a column by a butterfly, the block's waves in order).
__global__ void __launch_bounds__(MT) k_mix_grad(MixGeom g, int c0, int kc, const double* __restrict__ mu,
                                                 const double* __restrict__ sig, const double* __restrict__ gr,
                                                 const double* __restrict__ bt, double* __restrict__ part) {
    __shared__ double red[MT / 64][2][4][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kk = lane >> 4;
    const int ntiles = (g.rows + 16 * RT - 1) / (16 * RT);
    // per column tile t: u[t][0..3], meaning by the column's k (see above)
    double u[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int m = 0; m < 4; ++m) u[t][m] = 0.0;
    const double* b0p = bt + (size_t)i * g.n;
    const double* b1p = bt + (size_t)(16 + i) * g.n;
    for (int tile = blockIdx.x * (MT / 64) + wave; tile < ntiles; tile += gridDim.x * (MT / 64)) {
        const int row0 = tile * 16 * RT;
        v4d d[RT][2];
        const double* ap[RT];
        bool okr[RT];
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            d[q][0] = d[q][1] = v4d{0.0, 0.0, 0.0, 0.0};
            const int row = row0 + 16 * q + i;
            okr[q] = row < g.rows;
            ap[q] = gr + (size_t)(okr[q] ? row : 0) * g.n;
        }
        // lane (i, kk) takes x = k0 + 4 kk + s in MFMA step s: A[i][.] and B[.][col] agree.
        // The next chunk's operands are loaded while the current chunk's MFMAs run.
        double a[RT][4], b0[4], b1[4];
        {
            const int kb = 4 * kk, lim = g.n - kb;
#pragma unroll
            for (int q = 0; q < RT; ++q) load4(ap[q] + kb, okr[q] ? lim : 0, a[q]);
            load4(b0p + kb, lim, b0);
            load4(b1p + kb, lim, b1);
        }
        for (int k0 = 0; k0 < g.n; k0 += 16) {
            double an[RT][4], b0n[4], b1n[4];
            {
                const int kb = k0 + 16 + 4 * kk, lim = g.n - kb;
#pragma unroll
                for (int q = 0; q < RT; ++q) load4(ap[q] + kb, okr[q] ? lim : 0, an[q]);
                load4(b0p + kb, lim, b0n);
                load4(b1p + kb, lim, b1n);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int q = 0; q < RT; ++q) {
                    d[q][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][s], b0[s], d[q][0], 0, 0, 0);
                    d[q][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][s], b1[s], d[q][1], 0, 0, 0);
                }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
#pragma unroll
                for (int q = 0; q < RT; ++q) a[q][s] = an[q][s];
                b0[s] = b0n[s];
                b1[s] = b1n[s];
            }
        }
    // lane (i, kk) holds Y[row0 + 16 q + kk + 4 r][16 t + i]
#pragma unroll
        for (int q = 0; q < RT; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + 16 * q + kk + 4 * r;
                if (row >= g.rows) continue;
                int y, z;
                row_yz(g, row, y, z);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int col = 16 * t + i, cc = col / 3, k = col % 3;
                    if (cc >= kc) continue;
                    const int c = c0 + cc;
                    const double dy = g.x0[1] + y * g.h[1] - mu[c * g.d + 1];
                    const double dz = g.d == 3 ? g.x0[2] + z * g.h[2] - mu[c * g.d + 2] : 0.0;
                    const double f = exp(-(dy * dy + dz * dz) / (sig[c] * sig[c]));
                    const double fy = f * d[q][t][r];
                    u[t][0] += fy;
                    if (k == 0) {
                        u[t][1] += fy * dy;
                        u[t][2] += fy * dz;
                        u[t][3] += fy * (dy * dy + dz * dz);
                    }
                }
            }
    }
    // the four lanes of each column (kk = 0..3), then the block's waves in order
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double v = u[t][m];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (kk == 0) red[wave][t][m][i] = v;
        }
    __syncthreads();
    if (threadIdx.x < BC) {
        const int t = threadIdx.x / 16, col = threadIdx.x, cc = col / 3, k = col % 3;
        double v[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            v[m] = red[0][t][m][col % 16];
#pragma unroll
            for (int w = 1; w < MT / 64; ++w) v[m] += red[w][t][m][col % 16];
        }
        if (cc < CH) {
            double* o = part + (size_t)blockIdx.x * NS * CH + NS * cc;
            if (k == 0) {
                o[0] = v[0];
                o[2] = v[1];
                o[3] = v[2];
            } else if (k == 1) {
                o[1] = v[0];
            }
        }
    }
    __syncthreads();
    // R = (f q Y0 from the k = 0 column) + (f Y2 from the k = 2 column), in that order
    if (threadIdx.x < CH) {
        const int cc = threadIdx.x, c0l = 3 * cc, c2l = 3 * cc + 2;
        double r0 = red[0][c0l / 16][3][c0l % 16], r2 = red[0][c2l / 16][0][c2l % 16];
#pragma unroll
        for (int w = 1; w < MT / 64; ++w) {
            r0 += red[w][c0l / 16][3][c0l % 16];
            r2 += red[w][c2l / 16][0][c2l % 16];
        }
        part[(size_t)blockIdx.x * NS * CH + NS * cc + 4] = r0 + r2;
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
size_t mixture_partial_doubles() { return (size_t)GRAD_GRID * NS * CH + (size_t)MAX_ROW * BC; }
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
    if (g.n > MAX_ROW) return gsapi::fail(GS_ERR_UNSUPPORTED_SIZE, "mixture gradient: rows of at most 2048 points");
    const int ntiles = (g.rows + 16 * RT - 1) / (16 * RT);
    const int grid = std::min(GRAD_GRID, (ntiles + MT / 64 - 1) / (MT / 64));
    double* const bt = p->mixpart + (size_t)GRAD_GRID * NS * CH;
    for (int c0 = 0; c0 < K; c0 += CH) {
        const int kc = std::min(CH, K - c0);
        k_mix_table<<<(g.n * BC + MT - 1) / MT, MT, 0, p->stream>>>(g, c0, kc, mu, sigma, bt);
        k_mix_grad<<<grid, MT, 0, p->stream>>>(g, c0, kc, mu, sigma, g_dev, bt, p->mixpart);
        k_mix_grad_finish<<<NS * CH, MT, 0, p->stream>>>(g.d, K, c0, kc, grid, scale, a, sigma, p->mixpart, out_dev);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return gsapi::hip_fail(e, "mixture gradient launch");
    return GS_OK;
}

}  // extern "C"
