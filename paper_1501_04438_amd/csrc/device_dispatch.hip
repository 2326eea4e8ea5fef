// device_dispatch.hip -- size dispatch of the evaluation passes and the
// spectrum-assembly launcher.
#include <algorithm>

#include "assembly.hpp"
#include "device_api.hpp"
#include "sizes.hpp"

namespace gsk {

#define GS_DECL(N)                                                   \
    hipError_t launch_eval_##N(const EvalArgs&, hipStream_t, int);   \
    hipError_t launch_eval_g_##N(const EvalArgs&, hipStream_t, int); \
    int tile_variants_##N();
GS_SIZE_LIST(GS_DECL)
#undef GS_DECL

static bool cubic(const EvalArgs& a) {
    return a.nx == a.n && a.ny == a.n && (a.d == 2 || a.nz == a.n);
}

int energy_pencils(int d, int nx, int ny) { return d == 3 ? (nx + 1) * 2 * ny : nx + 1; }

// One pass of a rectangular grid at the length of the axis it transforms.
static hipError_t launch_pass_g(const EvalArgs& a, hipStream_t s, int pass) {
    const int len = (pass == 1 || pass == 5) ? a.nx : (pass == 3 && a.d == 3) ? a.nz : a.ny;
    switch (len) {
#define GS_CASE(N) \
    case N: return launch_eval_g_##N(a, s, pass);
        GS_SIZE_LIST(GS_CASE)
#undef GS_CASE
        default: return hipErrorInvalidValue;
    }
}

// One block: thread t sums part[t], part[t + 256], ... in order, then the fixed-order block
// sum; the same bits on every run.  The loads are issued eight at a time (the additions keep
// their order; a missing term adds 0).
__global__ void __launch_bounds__(256) k_energy_finish(const double* __restrict__ part, int count, double scale,
                                                       double* __restrict__ energy) {
    __shared__ double red[4];
    double v = 0.0;
    for (int i0 = threadIdx.x; i0 < count; i0 += 8 * 256) {
        double q[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) q[k] = (i0 + 256 * k < count) ? part[i0 + 256 * k] : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) v += q[k];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) energy[0] = scale * (((red[0] + red[1]) + red[2]) + red[3]);
}

hipError_t launch_energy_finish(const double* part, int count, double scale, double* energy, hipStream_t s) {
    k_energy_finish<<<1, 256, 0, s>>>(part, count, scale, energy);
    return hipGetLastError();
}

// First stage of the energy total over many partial sums: block b sums part[b chunk ..
// (b + 1) chunk) as k_energy_finish does (thread order, then the waves in order) into out[b].
__global__ void __launch_bounds__(256) k_energy_chunks(const double* __restrict__ part, int count, int chunk,
                                                       double* __restrict__ out) {
    __shared__ double red[4];
    const int b0 = blockIdx.x * chunk, b1 = min(count, b0 + chunk);
    double v = 0.0;
    for (int i0 = b0 + (int)threadIdx.x; i0 < b1; i0 += 8 * 256) {
        double q[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) q[k] = (i0 + 256 * k < b1) ? part[i0 + 256 * k] : 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) v += q[k];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

constexpr int kEnergyChunks = 256;

int energy_total_scratch() { return kEnergyChunks; }

hipError_t launch_energy_total(double* part, int count, double scale, double* energy, hipStream_t s) {
    if (count <= 4096) return launch_energy_finish(part, count, scale, energy, s);
    const int nb = std::min(kEnergyChunks, (count + 4095) / 4096);
    const int chunk = (count + nb - 1) / nb;
    double* sums = part + count;
    k_energy_chunks<<<nb, 256, 0, s>>>(part, count, chunk, sums);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_energy_finish(sums, nb, scale, energy, s);
}

// One thread per point of a row of the transform grid (blockIdx.y = y, blockIdx.z = z).
__global__ void __launch_bounds__(256) k_pad_embed(const double* __restrict__ rho, double* __restrict__ E,
                                                   int nx, int ny, int nz, int Nx, int Ny) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= Nx) return;
    double v = 0.0;
    if (x < nx && y < ny && z < nz) v = rho[((size_t)z * ny + y) * nx + x];
    E[((size_t)z * Ny + y) * Nx + x] = v;
}

// One thread per point of a row of the density's grid.
__global__ void __launch_bounds__(256) k_pad_crop(const double* __restrict__ E, double* __restrict__ u,
                                                  int nx, int ny, int Nx, int Ny) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= nx) return;
    u[((size_t)z * ny + y) * nx + x] = E[((size_t)z * Ny + y) * Nx + x];
}

hipError_t launch_pad_embed(const double* rho, double* E, int nx, int ny, int nz, int Nx, int Ny, int Nz,
                            hipStream_t s) {
    if (nx > Nx || ny > Ny || nz > Nz || Ny > 65535 || Nz > 65535) return hipErrorInvalidValue;
    k_pad_embed<<<dim3((Nx + 255) / 256, Ny, Nz), 256, 0, s>>>(rho, E, nx, ny, nz, Nx, Ny);
    return hipGetLastError();
}

hipError_t launch_pad_crop(const double* E, double* u, int nx, int ny, int nz, int Nx, int Ny, int Nz,
                           hipStream_t s) {
    if (nx > Nx || ny > Ny || nz > Nz || ny > 65535 || nz > 65535) return hipErrorInvalidValue;
    k_pad_crop<<<dim3((nx + 255) / 256, ny, nz), 256, 0, s>>>(E, u, nx, ny, Nx, Ny);
    return hipGetLastError();
}

hipError_t launch_eval(const EvalArgs& a, hipStream_t s, int which) {
    if (!cubic(a)) {
        for (int p = 1; p <= 5; ++p) {
            if (which >= 0 && which != p) continue;
            if (a.d == 2 && (p == 2 || p == 4)) continue;
            const hipError_t e = launch_pass_g(a, s, p);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    switch (a.n) {
#define GS_CASE(N) \
    case N: return launch_eval_##N(a, s, which);
        GS_SIZE_LIST(GS_CASE)
#undef GS_CASE
        default: return hipErrorInvalidValue;
    }
}

int tile_variants(int n) {
    switch (n) {
#define GS_CASE(N) \
    case N: return tile_variants_##N();
        GS_SIZE_LIST(GS_CASE)
#undef GS_CASE
        default: return 0;
    }
}

bool eval_size_supported(int d, int n) {
    if (d == 3 && n > GS_MAX_N_3D) return false;
    switch (n) {
#define GS_CASE(N) \
    case N: return true;
        GS_SIZE_LIST(GS_CASE)
#undef GS_CASE
        default: return false;
    }
}

int eval_sizes(int d, long long* out, int cap) {
    int c = 0;
#define GS_ADD(N)                                                   \
    if (!(d == 3 && N > GS_MAX_N_3D)) {                             \
        if (c < cap && out) out[c] = N;                             \
        ++c;                                                        \
    }
    GS_SIZE_LIST(GS_ADD)
#undef GS_ADD
    return c;
}

// Row blocks of 16 per wave: at most 9, with as few k1 chunks as possible.
static int assembly_mb(int n1) {
    const int blocks = (n1 + 15) / 16;
    const int chunks = (blocks + 8) / 9;
    return (blocks + chunks - 1) / chunks;
}

int assembly_ldk(int n1) {
    const int mb = assembly_mb(n1);
    const int chunks = ((n1 + 15) / 16 + mb - 1) / mb;
    return chunks * mb * 16;
}

template <int MB>
static hipError_t launch_mb(const AssemblyArgs& a, hipStream_t s) {
    const int n1b = a.n1b > 0 ? a.n1b : a.n1, n1c = a.n1c > 0 ? a.n1c : a.n1;
    const long ncols = (a.d == 3) ? (long)n1b * n1c : n1c;
    const int chunks = (a.n1 + MB * 16 - 1) / (MB * 16);
    dim3 grid((unsigned)((ncols + 63) / 64), chunks);
    if (a.d == 3)
        k_assemble<MB, 3><<<grid, 256, 0, s>>>(a.AT, a.FB, a.FC, a.ldk, a.n1, n1b, n1c, a.Qp, a.out, a.A0, a.c2,
                                               a.dxi[0], a.dxi[1], a.dxi[2], a.invM, a.dxx, a.lapu);
    else
        k_assemble<MB, 2><<<grid, 256, 0, s>>>(a.AT, a.FC, a.FC, a.ldk, a.n1, n1b, n1c, a.Qp, a.out, a.A0, a.c2,
                                               a.dxi[0], a.dxi[2], a.dxi[2], a.invM, a.dxx, a.lapu);
    return hipGetLastError();
}

// Loads the code object of the assembly kernel that launch_assembly(a) will run (a kernel's
// first launch in a process otherwise loads it on the host between the events that time it).
template <int MB>
static hipError_t load_mb(const AssemblyArgs& a) {
    hipFuncAttributes attr;
    return a.d == 3 ? hipFuncGetAttributes(&attr, (const void*)k_assemble<MB, 3>)
                    : hipFuncGetAttributes(&attr, (const void*)k_assemble<MB, 2>);
}

hipError_t load_assembly(const AssemblyArgs& a) {
    switch (assembly_mb(a.n1)) {
        case 1: return load_mb<1>(a);
        case 2: return load_mb<2>(a);
        case 3: return load_mb<3>(a);
        case 4: return load_mb<4>(a);
        case 5: return load_mb<5>(a);
        case 6: return load_mb<6>(a);
        case 7: return load_mb<7>(a);
        case 8: return load_mb<8>(a);
        case 9: return load_mb<9>(a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_assembly(const AssemblyArgs& a, hipStream_t s) {
    switch (assembly_mb(a.n1)) {
        case 1: return launch_mb<1>(a, s);
        case 2: return launch_mb<2>(a, s);
        case 3: return launch_mb<3>(a, s);
        case 4: return launch_mb<4>(a, s);
        case 5: return launch_mb<5>(a, s);
        case 6: return launch_mb<6>(a, s);
        case 7: return launch_mb<7>(a, s);
        case 8: return launch_mb<8>(a, s);
        case 9: return launch_mb<9>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gsk
