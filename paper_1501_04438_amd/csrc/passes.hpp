// passes.hpp -- the evaluation passes of the Gaussian-sum convolution on gfx950.
//
// The evaluation is one aperiodic convolution, u = (1/M) crop(IDFT(S . DFT(pad rho)))
// on the grid zero-padded from n to 2n points per axis (Section 2.2 with the
// padding of its Remark; the Taylor terms A0 rho + c2 Lap rho of Section 2.3 are
// folded into the stored spectrum S, which also carries 1/M).  Pruned passes,
// 3D (arrays C-ordered, x fastest; complex FP64):
//
//   P1 x_r2c : rho[z][y][x] (real)      -> X1[z][kx][y],  kx = 0..n   (two real rows per FFT)
//   P2 y_fwd : X1[z][kx][y]             -> X2[kx][ky][z], ky = 0..2n-1
//   P3 fused : X2[kx][ky][z] -> forward z (n -> 2n), * S[kx][|ky|][|kz|], inverse z
//              (2n -> n), in place
//   P4 y_inv : X2[kx][ky][z]            -> X1[z][kx][y]   (2n -> n)
//
// P2-P4 can run slab by slab over kx (kx0 .. kx0 + slab - 1), X2 then holding one
// slab: a cap on workspace memory for large n.
//   P5 x_c2r : X1[z][kx][y]             -> u[z][y][x]     (Hermitian n+1 -> 2n real -> n)
//
// 2D is P1, P3 along y on X1[kx][y] with S[kx][|ky|], and P5.  Every pass reads
// its input once and writes its output once; the zero padding is never stored.
// Each pass that changes the contiguous axis does so through the LDS exchange of
// its FFT: the first stage runs with the load-side thread mapping, the later
// stages with the store-side mapping, so both global sides move 256-byte runs.
#pragma once

#include "fft_core.hpp"
#include "sizes.hpp"

namespace gsk {

// spectrum mode of the fused pass
enum { SPEC_PLAIN = 0, SPEC_DIPOLAR = 1 };

struct DipoleArgs {
    double dxi[3];       // pi / (2 L_j) of the x, y, z axes: xi_k = k * dxi[j]
    double cdiag[3];     // 3 n_i m_i                    (x, y, z)
    double ccross[3];    // 3 (n_i m_j + n_j m_i)        (xy, xz, yz)
    double nm_over_M;    // (n.m) / (2n)^3
};

// Cache hints of the passes.  Bit 0: non-temporal loads of the streamed input (read
// once), bit 1: non-temporal stores of the output, bit 2 (fused pass): non-temporal
// spectrum loads.  Non-temporal accesses keep streamed data from displacing lines
// that are still useful; on MI355X they raise a plain copy from about 5.9 to 7 TB/s.
template <bool NT, class T> __device__ __forceinline__ T ldg(gp<const T> p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, class T> __device__ __forceinline__ void stg(gp<T> p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
// Each pass is compiled with these hints and without (plain accesses); the launch picks per
// pass (hint bits of the plan, default: hints for P1, P2, P4, P5 and plain P3, chosen by
// measurement at n = 256 over whole five-pass chains): non-temporal loads where the input is
// streamed once (P1, P4; P3's variant), non-temporal stores where the output is scattered in
// short runs (P2) or real (P5); P5 keeps its loads cached because each Hermitian row is read
// twice (direct and mirrored), and the fused pass its spectrum loads, because the +ky and
// -ky pencils of a block read the same row
constexpr int NT_P1 = 1, NT_P2 = 2, NT_P3 = 1, NT_P4 = 1, NT_P5 = 2;

// ---------------------------------------------------------------------------
// Launch geometry per transform length.
// ---------------------------------------------------------------------------
// Exchanges the upper 32 lanes of a with the lower 32 lanes of b (all four words).
__device__ __forceinline__ void swap_halves(cpx& a, cpx& b) {
    unsigned* pa = reinterpret_cast<unsigned*>(&a);
    unsigned* pb = reinterpret_cast<unsigned*>(&b);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(pa[i], pb[i], false, false);
        pa[i] = r[0];
        pb[i] = r[1];
    }
}

// Geometry of the fused pass on radix plan RV (FusedPlan): values and threads per
// half-transform, LDS area, pencils per block.
template <int N, int RV = 0> struct GeoZ {
    using FZ = FusedPlan<N, RV>;
    static constexpr int EZ = FZ::E, GZ = FZ::G, AZ = LdsAreaOf<FZ>::size;
    static constexpr int PPZ = (2 * GZ >= 128) ? 1 : 128 / (2 * GZ);
    static constexpr int TZ = PPZ * 2 * GZ;
};

template <int N> struct Geo {
    using F = FftCfg<N>;          // transforms of the x and y passes
    using FZ = FftCfgFused<N>;    // transforms of the fused pass (default radix plan)
    static constexpr int E = F::E, G = F::G, A = LdsArea<N>::size;
    static constexpr int EZ = FZ::E, GZ = FZ::G, AZ = LdsAreaOf<FZ>::size;
    // P1/P5: pairs of real rows per block (2*PPX rows of y, 16-byte complex each)
    // (at n = 2048 two pairs per block, not one: the transposed X1 accesses then move 64-byte
    // runs instead of 32-byte ones; measured 0.069 -> 0.039 ms for the 2D x-inverse)
    static constexpr int PPX = (N <= 256) ? 8 : (N <= 512 ? 4 : 2);
    // P2/P4: z-pencils per block
    static constexpr int PPY = (N <= 256) ? 16 : 8;
    // P3: pencils per block (two half-transforms each)
    static constexpr int PPZ = (2 * GZ >= 128) ? 1 : 128 / (2 * GZ);
    static constexpr int TX = PPX * G, TY = PPY * G, TZ = PPZ * 2 * GZ;
};

// Transforms of the x passes on radix plan XV (XPlan): values and threads per row transform
// (rows per block and LDS area as in Geo).
template <int N, int XV = 0> struct GeoX {
    using F = XPlan<N, XV>;
    static constexpr int E = F::E, G = F::G;
};

// Extents of a grid whose axes have their own n (x, y, z; 2D: z = 1).  A pass compiled with
// CUBE = true takes every extent as its transform length N (compile time) and ignores these;
// with CUBE = false the extents of the axes it does not transform come from here, and every
// row and pencil is bounds-checked.
struct Ext {
    int nx = 0, ny = 0, nz = 0;
};

// ---------------------------------------------------------------------------
// P1: x-direction real-to-complex of zero-padded rows.  Block = one z, 2*PPX rows.
// Two real rows a, b form c = a + i b; its padded transform C is split into the
// Hermitian spectra A = (C[m] + conj C[2n-m])/2, B = (C[m] - conj C[2n-m])/(2i).
// ---------------------------------------------------------------------------
// PX: row pairs per block (a tile-shape variant; the pairing of rows is the same for every PX,
// so every variant computes the same bits)
// RL: the rows are loaded again for the second half instead of being kept in registers across
// both (same values, same bits; E fewer complex values live through the first half's transform,
// which the batched kernels, sized for every length at once, need for their occupancy)
// XV: radix plan of the row transforms (XPlan).
// EMB (with CUBE): the density is the first ext.nx x ext.ny x ext.nz points of the transform
// grid, read from an array of those extents, zeros elsewhere (padding to B_3 without a copy).
template <int N, int NT = NT_P1, bool CUBE = true, int PX = Geo<N>::PPX, bool RL = false, int XV = 0,
          bool EMB = false>
__device__ __forceinline__ void x_r2c_tile(gp<const double> __restrict__ rho, gp<cpx> __restrict__ X1,
                                           gp<const cpx> __restrict__ tw, int bx, int z, int tid, bool active,
                                           cpx* lds, Ext ext = Ext()) {
    using Gm = Geo<N>;
    using Fx = typename GeoX<N, XV>::F;
    constexpr int E = Fx::E, G = Fx::G, PP = PX, A = Gm::A;
    const int NY = CUBE ? N : ext.ny;          // rows (y) of a plane
    const int tA = tid % G, pA = tid / G;      // load role: consecutive x
    const int pB = tid % PP, tB = tid / PP;    // store role: consecutive y
    const int y0 = bx * 2 * PP;
    // rows beyond n exist only when 2 PPX does not divide n
    constexpr bool FULL = CUBE && (N % (2 * PP) == 0);
    const bool okA = active && (FULL || (y0 + 2 * pA) < NY), okB = active && (FULL || (y0 + 2 * pB) < NY);
    // the two real rows of pair p: y0 + 16 (p / 8) + p % 8 and 8 rows further when the tile
    // divides the grid and holds a multiple of 8 pairs (each 16-byte store instruction on the
    // transposed X1 side then fills whole 128-byte lines: P1 at 256^3 0.0765 -> 0.0706 ms),
    // else y0 + 2p and y0 + 2p + 1
    // (the pairing follows the default tile, Geo<N>::PPX pairs, for every PX: the same bits)
    constexpr bool SPLIT = FULL && Gm::PPX % 8 == 0 && PP % 8 == 0;
    constexpr int RS = SPLIT ? 8 : 1;
    const int rowA = SPLIT ? y0 + 16 * (pA / 8) + pA % 8 : y0 + 2 * pA;
    const int rowB = SPLIT ? y0 + 16 * (pB / 8) + pB % 8 : y0 + 2 * pB;

    cpx x[RL ? 1 : E];
    if constexpr (EMB) {
        static_assert(CUBE && !RL, "embedded density on the cubic tiles");
        const bool r0 = okA && z < ext.nz && rowA < ext.ny, r1 = okA && z < ext.nz && rowA + RS < ext.ny;
        gp<const double> ra = rho + ((size_t)z * ext.ny + rowA) * ext.nx;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = tA + G * e;
            const bool in = j < ext.nx;
            x[e] = cmk(r0 && in ? ldg<NT & 1>(ra + j) : 0.0, r1 && in ? ldg<NT & 1>(ra + (size_t)RS * ext.nx + j) : 0.0);
        }
    } else if constexpr (!RL) {
        gp<const double> ra = rho + ((size_t)z * NY + rowA) * N;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = tA + G * e;
            x[e] = okA ? cmk(ldg<NT & 1>(ra + j), ldg<NT & 1>(ra + (size_t)RS * N + j)) : cmk(0.0, 0.0);
        }
    }
    gp<cpx> out = X1 + (size_t)z * (N + 1) * NY + rowB;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cpx v[E];
        if constexpr (RL) {
            const double* rb = (const double*)rho;
            // an opaque base for the second load, so that it is not merged with the first
            if (h) asm volatile("" : "+s"(rb));
            gp<const double> ra = (gp<const double>)rb + ((size_t)z * NY + rowA) * N;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = tA + G * e;
                v[e] = okA ? cmk(ldg<NT & 1>(ra + j), ldg<NT & 1>(ra + (size_t)RS * N + j)) : cmk(0.0, 0.0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = x[e];
        }
        // the separate twist measured faster here than the twisted roots (its h = 1 roots
        // of the 16 x 16 plan double the stage-2 power products in the unrolled h loop)
        if (h) twist_in<Fx>(v, tA, tw);
        fft<Fx, false>(v, tA, lds + pA * A, tB, lds + pB * A, tw);
        lds_barrier();
#pragma unroll
        for (int e = 0; e < E; ++e) lds[pB * A + lds_pad(tB + G * e)] = v[e];
        lds_barrier();
        // k = tB + G e is below n/2 for e < E/2 (kept by both halves); at e = E/2 it is
        // n/2 + tB, kept only by the even half's thread tB = 0; beyond it is never kept
#pragma unroll
        for (int e = 0; e <= E / 2; ++e) {
            if (e == E / 2 && !(h == 0 && tB == 0)) continue;
            const int k = tB + G * e;
            if (okB) {
                const int kp = h ? (N - 1 - k) : ((N - k) % N);
                const cpx zk = v[e], zp = lds[pB * A + lds_pad(kp)];
                const cpx sa = cmk(0.5 * (zk.x + zp.x), 0.5 * (zk.y - zp.y));       // (Z + conj P)/2
                const cpx df = cmk(zk.x - zp.x, zk.y + zp.y);                        //  Z - conj P
                const cpx sb = cmk(0.5 * df.y, -0.5 * df.x);                         // /(2i)
                const int m = 2 * k + h;
                gp<cpx> o = out + (size_t)m * NY;
                stg<(NT & 2) != 0>(o, sa);
                stg<(NT & 2) != 0>(o + RS, sb);
            }
        }
        lds_barrier();
    }
}

// At n = 2048 the compiler's own allocation takes 256 VGPRs + 42 accumulator registers (one wave
// per SIMD); capped at two waves per SIMD it spills 172 bytes per lane and still runs faster
// (measured 0.038 -> 0.033 ms for 2D 2048^2; the same cap slows the x-inverse and n = 1024).
template <int N, int NT = NT_P1, int PX = Geo<N>::PPX, int XV = 0>
__global__ void __launch_bounds__((PX * GeoX<N, XV>::G)) __attribute__((amdgpu_waves_per_eu(N == 2048 ? 2 : 1)))
k_x_r2c(const double* __restrict__ rho, cpx* __restrict__ X1,
                                                      const cpx* __restrict__ tw) {
    __shared__ cpx lds[PX * Geo<N>::A];
    x_r2c_tile<N, NT, true, PX, false, XV>((gp<const double>)rho, (gp<cpx>)X1, (gp<const cpx>)tw, blockIdx.x,
                                           blockIdx.y, threadIdx.x, true, lds);
}

// ---------------------------------------------------------------------------
// P5: x-direction complex-to-real with cropping.  Inverse of P1 (unnormalised).
// ---------------------------------------------------------------------------
// SC: the outputs are stored times oscale (the rho gradient of the energy, cell u).
// EMB (with CUBE): the potential is stored for the first ext.nx x ext.ny x ext.nz points of the
// transform grid only, into an array of those extents (padding to B_3 without a copy).
template <int N, int NT = NT_P5, bool SC = false, bool CUBE = true, int PX = Geo<N>::PPX, int XV = 0,
          bool EMB = false>
__device__ __forceinline__ void x_c2r_tile(gp<const cpx> __restrict__ X1, gp<double> u,
                                           gp<const cpx> __restrict__ tw, int bx, int z, int tid, bool active,
                                           cpx* lds, Ext ext = Ext(), double oscale = 1.0) {
    using Gm = Geo<N>;
    using Fx = typename GeoX<N, XV>::F;
    constexpr int E = Fx::E, G = Fx::G, PP = PX, A = Gm::A;
    const int NY = CUBE ? N : ext.ny;          // rows (y) of a plane
    const int tA = tid % G, pA = tid / G;      // store role: consecutive x
    const int pB = tid % PP, tB = tid / PP;    // load role: consecutive y
    const int y0 = bx * 2 * PP;
    // rows beyond n exist only when 2 PPX does not divide n
    constexpr bool FULL = CUBE && (N % (2 * PP) == 0);
    const bool okA = active && (FULL || (y0 + 2 * pA) < NY), okB = active && (FULL || (y0 + 2 * pB) < NY);
    // rows of pair p as in x_r2c_tile (8 rows apart in groups of 16 when the tile divides the
    // grid and holds a multiple of 8 pairs: whole 128-byte lines per load instruction on the
    // transposed X1 side)
    constexpr bool SPLIT = FULL && Gm::PPX % 8 == 0 && PP % 8 == 0;
    constexpr int RS = SPLIT ? 8 : 1;
    const int rowA = SPLIT ? y0 + 16 * (pA / 8) + pA % 8 : y0 + 2 * pA;
    const int rowB = SPLIT ? y0 + 16 * (pB / 8) + pB % 8 : y0 + 2 * pB;
    gp<const cpx> in = X1 + (size_t)z * (N + 1) * NY + rowB;

    cpx acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = cmk(0.0, 0.0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cpx v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int m = 2 * (tB + G * e) + h;       // padded index 0..2n-1
            const bool direct = m <= N;
            const int mm = direct ? m : 2 * N - m;
            cpx a = cmk(0.0, 0.0), b = cmk(0.0, 0.0);
            if (okB) {
                gp<const cpx> p = in + (size_t)mm * NY;
                a = ldg<NT & 1>(p);
                b = ldg<NT & 1>(p + RS);
            }
            if (!direct) { a.y = -a.y; b.y = -b.y; }
            v[e] = cmk(a.x - b.y, a.y + b.x);          // a + i b
        }
        fft_t<Fx, true>(v, tA, lds + pA * A, tB, lds + pB * A, tw, h);   // cropping twist included
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = cadd(acc[e], v[e]);
        lds_barrier();
    }
    if constexpr (EMB) {
        static_assert(CUBE, "embedded potential on the cubic tiles");
        const bool r0 = okA && z < ext.nz && rowA < ext.ny, r1 = okA && z < ext.nz && rowA + RS < ext.ny;
        gp<double> ua = u + ((size_t)z * ext.ny + rowA) * ext.nx;
        if constexpr (SC) {
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = cscale(acc[e], oscale);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = tA + G * e;
            if (j < ext.nx) {
                if (r0) stg<(NT & 2) != 0>(ua + j, acc[e].x);
                if (r1) stg<(NT & 2) != 0>(ua + (size_t)RS * ext.nx + j, acc[e].y);
            }
        }
    } else if (okA) {
        const size_t o = ((size_t)z * NY + rowA) * N;
        gp<double> ua = u + o;
        if constexpr (SC) {
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = cscale(acc[e], oscale);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = tA + G * e;
            stg<(NT & 2) != 0>(ua + j, acc[e].x);
            stg<(NT & 2) != 0>(ua + (size_t)RS * N + j, acc[e].y);
        }
    }
}

// P5 of a cubic grid with the two halves of the padded inverse (h = 0, 1) on the two 32-lane
// halves of every wave: each thread loads and transforms one half, once (x_c2r_tile loads
// and transforms both halves in turn), and the halves' sum is formed by a lane swap, each
// lane then storing half of the pair's outputs (E/2 values of each row).  The same sums in
// the same order as x_c2r_tile, so the same bits; two LDS areas per row pair.  For the
// tiles whose PX G threads per half fill whole half-waves.  The outputs are stored times
// oscale with SC, as x_c2r_tile does.
// Decided per length, so that every tile shape of a length (PPX and 2 PPX row pairs) has the
// same layout: the default tile fills whole half-waves and the doubled tile's two LDS areas
// per pair fit in the 160 KiB of a CU.
template <int N, int XV = 0> constexpr bool p5_split_len() {
    return (Geo<N>::PPX * GeoX<N, XV>::G) % 32 == 0 && 2 * 2 * Geo<N>::PPX * Geo<N>::A * 16 <= 160 * 1024;
}
template <int N, int PX, int XV = 0> constexpr bool p5_split() {
    return p5_split_len<N, XV>() && (PX * GeoX<N, XV>::G) % 32 == 0 && 2 * PX * GeoX<N, XV>::G <= 1024;
}
template <int N, int PX, int XV = 0> constexpr int p5_threads() {
    return (p5_split<N, PX, XV>() ? 2 : 1) * PX * GeoX<N, XV>::G;
}

template <int N, int NT, bool SC, int PX, int XV = 0, bool EMB = false>
__device__ __forceinline__ void x_c2r_tile_split(gp<const cpx> __restrict__ X1, gp<double> u,
                                                 gp<const cpx> __restrict__ tw, int bx, int z, int tid, cpx* lds,
                                                 double oscale, bool active = true, Ext ext = Ext()) {
    using Gm = Geo<N>;
    using Fx = typename GeoX<N, XV>::F;
    constexpr int E = Fx::E, G = Fx::G, PP = PX, A = Gm::A;
    static_assert(p5_split<N, PX, XV>(), "whole half-waves");
    const int w = tid >> 6, l = tid & 63, h = l >> 5;
    const int tq = 32 * w + (l & 31);           // thread within its half
    const int tA = tq % G, pA = tq / G;         // store role: consecutive x
    const int pB = tq % PP, tB = tq / PP;       // load role: consecutive y
    const int y0 = bx * 2 * PP;
    constexpr bool FULL = (N % (2 * PP) == 0);
    const bool okA = active && (FULL || (y0 + 2 * pA) < N), okB = active && (FULL || (y0 + 2 * pB) < N);
    constexpr bool SPLIT = FULL && Gm::PPX % 8 == 0 && PP % 8 == 0;
    constexpr int RS = SPLIT ? 8 : 1;
    const int rowA = SPLIT ? y0 + 16 * (pA / 8) + pA % 8 : y0 + 2 * pA;
    const int rowB = SPLIT ? y0 + 16 * (pB / 8) + pB % 8 : y0 + 2 * pB;
    gp<const cpx> in = X1 + (size_t)z * (N + 1) * N + rowB;
    cpx v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int m = 2 * (tB + G * e) + h;           // padded index 0..2n-1
        const bool direct = m <= N;
        const int mm = direct ? m : 2 * N - m;
        cpx a = cmk(0.0, 0.0), b = cmk(0.0, 0.0);
        if (okB) {
            gp<const cpx> p = in + (size_t)mm * N;
            a = ldg<NT & 1>(p);
            b = ldg<NT & 1>(p + RS);
        }
        if (!direct) { a.y = -a.y; b.y = -b.y; }
        v[e] = cmk(a.x - b.y, a.y + b.x);              // a + i b
    }
    fft_t<Fx, true>(v, tA, lds + (h * PP + pA) * A, tB, lds + (h * PP + pB) * A, tw, h);
    // EMB: only the first ext.nx x ext.ny x ext.nz points, into an array of those extents
    const int OX = EMB ? ext.nx : N, OY = EMB ? ext.ny : N;
    const bool r0 = okA && (!EMB || (z < ext.nz && rowA < ext.ny));
    const bool r1 = okA && (!EMB || (z < ext.nz && rowA + RS < ext.ny));
    gp<double> ua = u + ((size_t)z * OY + rowA) * OX;
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        // lanes h = 0 end with the sum for element e, lanes h = 1 with that for e + E/2
        cpx a = v[e], b = v[e + E / 2];
        swap_halves(a, b);
        cpx r = cadd(a, b);
        const int j = tA + G * (h * (E / 2) + e);
        if (EMB ? (r0 || r1) && j < ext.nx : okA) {
            if constexpr (SC) r = cscale(r, oscale);
            if (!EMB || r0) stg<(NT & 2) != 0>(ua + j, r.x);
            if (!EMB || r1) stg<(NT & 2) != 0>(ua + (size_t)RS * OX + j, r.y);
        }
    }
}

// P5; SC: the outputs stored times oscale (the energy's rho gradient cell u; the energy
// itself is summed by the fused pass).
template <int N, int NT = NT_P5, int PX = Geo<N>::PPX, bool SC = false, int XV = 0>
__global__ void __launch_bounds__((p5_threads<N, PX, XV>())) k_x_c2r(const cpx* __restrict__ X1, double* __restrict__ u,
                                                                   const cpx* __restrict__ tw, double oscale = 1.0) {
    if constexpr (p5_split<N, PX, XV>()) {
        __shared__ cpx lds[2 * PX * Geo<N>::A];
        x_c2r_tile_split<N, NT, SC, PX, XV>((gp<const cpx>)X1, (gp<double>)u, (gp<const cpx>)tw, blockIdx.x,
                                            blockIdx.y, threadIdx.x, lds, oscale);
    } else {
        __shared__ cpx lds[PX * Geo<N>::A];
        x_c2r_tile<N, NT, SC, true, PX, XV>((gp<const cpx>)X1, (gp<double>)u, (gp<const cpx>)tw, blockIdx.x,
                                            blockIdx.y, threadIdx.x, true, lds, Ext(), oscale);
    }
}

// P1 and P5 of padding to B_3 on a cubic transform grid: the density (ext points per axis, in
// the first points of each axis) read, and the potential written, in place of copies into and
// out of a grid-sized array.
template <int N, int NT>
__global__ void __launch_bounds__(Geo<N>::TX) __attribute__((amdgpu_waves_per_eu(N == 2048 ? 2 : 1)))
k_x_r2c_emb(const double* __restrict__ rho, cpx* __restrict__ X1, const cpx* __restrict__ tw, Ext ext) {
    __shared__ cpx lds[Geo<N>::PPX * Geo<N>::A];
    x_r2c_tile<N, NT, true, Geo<N>::PPX, false, 0, true>((gp<const double>)rho, (gp<cpx>)X1, (gp<const cpx>)tw,
                                                         blockIdx.x, blockIdx.y, threadIdx.x, true, lds, ext);
}

template <int N, int NT, bool SC>
__global__ void __launch_bounds__((p5_threads<N, Geo<N>::PPX>())) k_x_c2r_emb(const cpx* __restrict__ X1,
                                                                              double* __restrict__ u,
                                                                              const cpx* __restrict__ tw, Ext ext,
                                                                              double oscale) {
    constexpr int PX = Geo<N>::PPX;
    if constexpr (p5_split<N, PX>()) {
        __shared__ cpx lds[2 * PX * Geo<N>::A];
        x_c2r_tile_split<N, NT, SC, PX, 0, true>((gp<const cpx>)X1, (gp<double>)u, (gp<const cpx>)tw, blockIdx.x,
                                                 blockIdx.y, threadIdx.x, lds, oscale, true, ext);
    } else {
        __shared__ cpx lds[PX * Geo<N>::A];
        x_c2r_tile<N, NT, SC, true, PX, 0, true>((gp<const cpx>)X1, (gp<double>)u, (gp<const cpx>)tw, blockIdx.x,
                                                 blockIdx.y, threadIdx.x, true, lds, ext, oscale);
    }
}

// ---------------------------------------------------------------------------
// P2: y-direction forward with zero padding.  Block = one kx, PPY consecutive z.
// ---------------------------------------------------------------------------
// PY: z-pencils per block (a tile-shape variant: the same bits for every PY)
// YV: radix plan of the pencil transforms (XPlan, as for the x passes)
template <int N, int NT = NT_P2, bool CUBE = true, int PY = Geo<N>::PPY, int YV = 0>
__device__ __forceinline__ void y_fwd_tile(gp<const cpx> __restrict__ X1, gp<cpx> __restrict__ X2,
                                           gp<const cpx> __restrict__ tw, int kx0, int bx, int kxl, int tid,
                                           bool active, cpx* lds, Ext ext = Ext()) {
    using Gm = Geo<N>;
    using Fy = typename GeoX<N, YV>::F;
    constexpr int E = Fy::E, G = Fy::G, PP = PY, A = Gm::A;
    const int NX = CUBE ? N : ext.nx, NZ = CUBE ? N : ext.nz;
    const int tA = tid % G, pA = tid / G;      // load role: consecutive y
    const int pB = tid % PP, tB = tid / PP;    // store role: consecutive z
    const int kx = kx0 + kxl;                         // slab-local and global kx
    const int z0 = bx * PP;
    // z beyond n exists only when PPY does not divide n
    constexpr bool FULL = CUBE && (N % PP == 0);
    const bool okA = active && (FULL || (z0 + pA) < NZ), okB = active && (FULL || (z0 + pB) < NZ);

    cpx x[E];
    {
        gp<const cpx> src = X1 + ((size_t)(z0 + pA) * (NX + 1) + kx) * N;
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = okA ? ldg<NT & 1>(src + tA + G * e) : cmk(0.0, 0.0);
    }
    gp<cpx> dst = X2 + (size_t)kxl * 2 * N * NZ + z0 + pB;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cpx v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = x[e];
        if (h) twist_const<Fy, false>(v);        // the rest of the twist rides in fft
        fft<Fy, false>(v, tA, lds + pA * A, tB, lds + pB * A, tw, h);
        if (okB) {
#pragma unroll
            for (int e = 0; e < E; ++e) stg<(NT & 2) != 0>(dst + (size_t)(2 * (tB + G * e) + h) * NZ, v[e]);
        }
        lds_barrier();
    }
}

template <int N, int NT = NT_P2, int PY = Geo<N>::PPY, int YV = 0>
__global__ void __launch_bounds__((PY * GeoX<N, YV>::G)) k_y_fwd(const cpx* __restrict__ X1, cpx* __restrict__ X2,
                                                                const cpx* __restrict__ tw, int kx0) {
    __shared__ cpx lds[PY * Geo<N>::A];
    y_fwd_tile<N, NT, true, PY, YV>((gp<const cpx>)X1, (gp<cpx>)X2, (gp<const cpx>)tw, kx0, blockIdx.x, blockIdx.y,
                                threadIdx.x, true, lds);
}

// ---------------------------------------------------------------------------
// P4: y-direction inverse with cropping.  Block = one kx, PPY consecutive z.
// ---------------------------------------------------------------------------
template <int N, int NT = NT_P4, bool CUBE = true, int PY = Geo<N>::PPY, int YV = 0>
__device__ __forceinline__ void y_inv_tile(gp<const cpx> __restrict__ X2, gp<cpx> __restrict__ X1,
                                           gp<const cpx> __restrict__ tw, int kx0, int bx, int kxl, int tid,
                                           bool active, cpx* lds, Ext ext = Ext()) {
    using Gm = Geo<N>;
    using Fy = typename GeoX<N, YV>::F;
    constexpr int E = Fy::E, G = Fy::G, PP = PY, A = Gm::A;
    const int NX = CUBE ? N : ext.nx, NZ = CUBE ? N : ext.nz;
    const int tA = tid % G, pA = tid / G;      // store role: consecutive y
    const int pB = tid % PP, tB = tid / PP;    // load role: consecutive z
    const int kx = kx0 + kxl;
    const int z0 = bx * PP;
    // z beyond n exists only when PPY does not divide n
    constexpr bool FULL = CUBE && (N % PP == 0);
    const bool okA = active && (FULL || (z0 + pA) < NZ), okB = active && (FULL || (z0 + pB) < NZ);
    gp<const cpx> src = X2 + (size_t)kxl * 2 * N * NZ + z0 + pB;

    cpx acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = cmk(0.0, 0.0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cpx v[E];
#pragma unroll
        for (int e = 0; e < E; ++e)
            v[e] = okB ? ldg<NT & 1>(src + (size_t)(2 * (tB + G * e) + h) * NZ) : cmk(0.0, 0.0);
        fft_t<Fy, true>(v, tA, lds + pA * A, tB, lds + pB * A, tw, h);   // cropping twist included
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = cadd(acc[e], v[e]);
        lds_barrier();
    }
    if (okA) {
        gp<cpx> dst = X1 + ((size_t)(z0 + pA) * (NX + 1) + kx) * N;
#pragma unroll
        for (int e = 0; e < E; ++e) stg<(NT & 2) != 0>(dst + tA + G * e, acc[e]);
    }
}

template <int N, int NT = NT_P4, int PY = Geo<N>::PPY, int YV = 0>
__global__ void __launch_bounds__((PY * GeoX<N, YV>::G)) k_y_inv(const cpx* __restrict__ X2, cpx* __restrict__ X1,
                                                                const cpx* __restrict__ tw, int kx0) {
    __shared__ cpx lds[PY * Geo<N>::A];
    y_inv_tile<N, NT, true, PY, YV>((gp<const cpx>)X2, (gp<cpx>)X1, (gp<const cpx>)tw, kx0, blockIdx.x, blockIdx.y,
                                threadIdx.x, true, lds);
}

// ---------------------------------------------------------------------------
// P3: fused forward transform along the contiguous axis, multiplication by the
// stored spectrum (folded Taylor terms and 1/M included), inverse transform.
// Each pencil is carried by two thread groups: the even (h = 0) and the odd
// (h = 1) half of the padded spectrum.  DIM = 3: pencils X2[kx][ky][:],
// spectrum row S[kx][|ky|][:]; DIM = 2: pencils X1[kx][:], row S[kx][:].
//
// Lane roles: a pencil's G-thread halves sit at lanes l and l + 32 of the same waves
// (G <= 32: one wave; G = 128: four waves, each holding 32 threads of both halves), so the
// even/odd combination after the inverse is a cross-half lane swap (v_permlane32_swap) and
// an add, with no LDS round trip; at G = 64 each half fills one wave (its exchanges then
// need no block barrier) and the halves are combined through LDS.  Persistent: a block walks pencil groups
// g = blockIdx.x, + gridDim.x, ...  (No register prefetch: the registers it needs
// cost a wave per SIMD, which hides more latency than the prefetch did.)  In 3D
// the pencils of a kx plane are visited in the order ky = 0, n, 1, 2n-1, 2,
// 2n-2, ...: the two pencils +ky and -ky that share a spectrum row sit in the
// same block.
// ---------------------------------------------------------------------------
template <int N, int RV = 0> struct FusedRoles {
    static constexpr int G = GeoZ<N, RV>::GZ;
    // (G = 128: 2D n = 1024, 2048 and the 3D n = 1024 fused plan; the lane swap saves the
    // LDS round trip and two block barriers per pencil: 0.057 -> 0.055 ms at 2D 2048^2)
    static constexpr bool SWAP = (G <= 32) || (G % 128 == 0);
    // t: thread within its half-transform, h: half (0 even, 1 odd), pl: pencil in the block
    __device__ __forceinline__ static void get(int tid, int& t, int& h, int& pl) {
        if constexpr (G <= 32) {
            const int w = tid >> 6, l = tid & 63;
            h = l >> 5;
            t = l % G;
            pl = w * (32 / G) + (l & 31) / G;
        } else if constexpr (SWAP) {
            constexpr int WPP = G / 32;
            const int w = tid >> 6, l = tid & 63;
            h = l >> 5;
            pl = w / WPP;
            t = (w % WPP) * 32 + (l & 31);
        } else {
            t = tid % G;
            h = (tid / G) & 1;
            pl = tid / (2 * G);
        }
    }
};


// NY: the y extent (3D pencils X2[kx][ky][:], ky = 0..2 NY - 1)
template <int N, int DIM>
__device__ __forceinline__ int fused_pencil(int slot, int NY) {
    if constexpr (DIM == 2) {
        return slot;
    } else {
        const int kx = slot / (2 * NY), s = slot % (2 * NY);
        const int i = s >> 1;
        const int ky = (s == 0) ? 0 : (s == 1) ? NY : ((s & 1) ? 2 * NY - i : i);
        return kx * 2 * NY + ky;
    }
}

// 2D, long pencils: the pencils kx = 0 and kx = NX, both real along y (the x transform of real
// rows is real at its zero and Nyquist frequencies), ride in one complex pencil a + i b: one
// transform pair for both, so NX pencil slots instead of NX + 1 (at n = 1024 the launch is
// otherwise two whole rounds of co-resident blocks plus one block).  After the forward
// transform C = A + i B, the mirror W(m) = C(-m) separates the two spectra,
// A = (C + conj W) / 2 and i B = (C - conj W) / 2, which take their own spectrum rows S0 and
// SN; the inverse of S0 A + SN (i B) is the pair of real results a' + i b'.
// Taken where the plan holds 8 values per thread in 128-thread halves (2D n = 1024): there the
// packed path's registers fit beside the transform's (170 -> 192 VGPRs, two waves per SIMD
// either way); the 16-value plans have no room for it (n = 2048: one wave per SIMD instead of
// two).
template <int N, int DIM, int RV = 0> constexpr bool fused_pack() {
    return DIM == 2 && N >= 1024 && GeoZ<N, RV>::EZ <= 8 && GeoZ<N, RV>::GZ <= 128;
}
template <int N, int DIM, int RV = 0> __host__ __device__ constexpr int fused_slots(int npencils) {
    return fused_pack<N, DIM, RV>() ? npencils - 1 : npencils;
}

template <int N, int DIM>
__device__ __forceinline__ gp<const double> fused_row(gp<const double> spec, int pencil, int kx0, int NY) {
    if constexpr (DIM == 3) {
        const int kx = kx0 + pencil / (2 * NY), ky = pencil % (2 * NY);
        const int aky = ky <= NY ? ky : 2 * NY - ky;
        return spec + ((size_t)kx * (NY + 1) + aky) * (N + 1);
    } else {
        return spec + (size_t)pencil * (N + 1);
    }
}

template <int N, int DIM, int NT, int RV = 0>
__device__ __forceinline__ void fused_load(gp<const cpx> X, int pencil, bool ok, int t, cpx (&v)[GeoZ<N, RV>::EZ]) {
    constexpr int E = GeoZ<N, RV>::EZ, G = GeoZ<N, RV>::GZ;
    gp<const cpx> base = X + (size_t)pencil * N;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = ok ? ldg<NT & 1>(base + t + G * e) : cmk(0.0, 0.0);
}

// The packed pencil (fused_pack): the real parts of pencils 0 and NX as one complex pencil.
template <int N, int NT, int RV = 0>
__device__ __forceinline__ void fused_load_pair(gp<const cpx> X, int NX, int t, cpx (&v)[GeoZ<N, RV>::EZ]) {
    constexpr int E = GeoZ<N, RV>::EZ, G = GeoZ<N, RV>::GZ;
    gp<const cpx> b0 = X, bn = X + (size_t)NX * N;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cmk(ldg<NT & 1>(b0 + t + G * e).x, ldg<NT & 1>(bn + t + G * e).x);
}

template <int N, int DIM, int NT, int RV = 0>
__device__ __forceinline__ void fused_spec(gp<const double> spec, int pencil, int kx0, bool ok, int t, int h,
                                           double (&sv)[GeoZ<N, RV>::EZ], int NY) {
    constexpr int E = GeoZ<N, RV>::EZ, G = GeoZ<N, RV>::GZ;
    gp<const double> srow = fused_row<N, DIM>(spec, ok ? pencil : 0, kx0, NY);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int m = 2 * (t + G * e) + h;          // padded index along the pencil
        sv[e] = ok ? ldg<(NT & 4) != 0>(srow + (m <= N ? m : 2 * N - m)) : 0.0;
    }
}

// The energy sum of one pencil by Parseval's identity: with the folded spectrum S (1/M
// included) the potential is the inverse transform of S rho^, so sum_x rho u over the grid is
// sum_k S(k) |rho^(k)|^2 over the whole padded spectrum.  The x transform keeps kx = 0..NX of
// its 2 NX values; the spectrum is even in every axis, so each kept plane other than kx = 0
// and kx = NX stands for its mirror too (weight 2).  Each pencil's sum (acc over its threads,
// in a fixed order) goes to part[index of the pencil in the whole grid], so the bits do not
// depend on the launch shape.  Called by every thread of the block (for G > 32 a pencil's
// waves are summed through LDS behind block barriers).
template <int N, int DIM, int RV = 0>
__device__ __forceinline__ void fused_energy_store(double acc, bool ok, int pencil, int kx0, int t, int h, int pl,
                                                   int NX, int NY, gp<double> part) {
    constexpr int G = GeoZ<N, RV>::GZ;
    if constexpr (G <= 32) {
        // a pencil: G lanes in each 32-lane half of one wave
#pragma unroll
        for (int o = G / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
        acc += __shfl_xor(acc, 32, 64);
    } else {
        // a pencil: 2 G / 64 whole waves (one half each at G = 64, both halves at G = 128)
        static_assert((2 * G) % 64 == 0, "whole waves per pencil");
        constexpr int WP = 2 * G / 64;
        __shared__ double red[16];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (t == 0 && h == 0) {
            acc = red[pl * WP];
#pragma unroll
            for (int i = 1; i < WP; ++i) acc += red[pl * WP + i];
        }
        __syncthreads();
    }
    if (ok && t == 0 && h == 0) {
        const int kx = (DIM == 3) ? kx0 + pencil / (2 * NY) : pencil;
        const double w = (kx == 0 || kx == NX) ? 1.0 : 2.0;
        part[(DIM == 3 ? (size_t)kx0 * 2 * NY : 0) + pencil] = w * acc;
    }
}

// Transform, spectrum multiplication, inverse transform and even/odd combination
// of one pencil held in v (spectrum values in sv); stores the pencil if ok.  EN: also the
// pencil's energy sum into part (fused_energy_store).
template <int N, int DIM, int MODE, int NT = NT_P3, bool EN = false, int RV = 0>
__device__ __forceinline__ void fused_body(gp<cpx> __restrict__ X, gp<const cpx> __restrict__ tw, int pencil, int kx0,
                                           bool ok, const DipoleArgs& dip, int t, int h, int pl,
                                           cpx (&v)[GeoZ<N, RV>::EZ], const double (&sv)[GeoZ<N, RV>::EZ],
                                           cpx* lds, cpx* area, int NX, int NY, gp<double> part = nullptr) {
    using Gm = GeoZ<N, RV>;
    using FZ = typename Gm::FZ;
    constexpr int E = Gm::EZ, G = Gm::GZ, A = Gm::AZ;
    constexpr bool FW = (G <= 64), CW = (2 * G <= 64);
    // the odd half's padding twist rides in the transforms (fft, fft_t with h = 1)
    if (h) twist_const<FZ, false>(v);
    fft<FZ, false, FW>(v, t, area, t, area, tw, h);
    double acc = 0.0;
    if constexpr (MODE == SPEC_DIPOLAR) {
        // (n.xi)(m.xi) with Nyquist taken as 0 in the odd (cross) factors
        const int kx = (DIM == 3) ? kx0 + pencil / (2 * NY) : pencil;
        const int ky = (DIM == 3) ? pencil % (2 * NY) : 0;
        const double xe = kx * dip.dxi[0];
        const int sy = ky < NY ? ky : ky - 2 * NY;
        const double ye = sy * dip.dxi[1];
        const double xo = (kx == NX) ? 0.0 : xe;
        const double yo = (ky == NY) ? 0.0 : ye;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int m = 2 * (t + G * e) + h;
            const int sz = m < N ? m : m - 2 * N;
            const double ze = sz * dip.dxi[2];
            const double zo = (m == N) ? 0.0 : ze;
            const double f = dip.cdiag[0] * xe * xe + dip.cdiag[1] * ye * ye + dip.cdiag[2] * ze * ze +
                             dip.ccross[0] * xo * yo + dip.ccross[1] * xo * zo + dip.ccross[2] * yo * zo;
            const double s = f * sv[e] - dip.nm_over_M;
            if constexpr (EN) acc += s * (v[e].x * v[e].x + v[e].y * v[e].y);
            v[e] = cscale(v[e], s);
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (EN) acc += sv[e] * (v[e].x * v[e].x + v[e].y * v[e].y);
            v[e] = cscale(v[e], sv[e]);
        }
    }
    if constexpr (EN) fused_energy_store<N, DIM, RV>(acc, ok, pencil, kx0, t, h, pl, NX, NY, part);
    lds_sync<FW>();
    fft_t<FZ, true, FW>(v, t, area, t, area, tw, h);
    gp<cpx> base = X + (size_t)pencil * N;
    if constexpr (FusedRoles<N, RV>::SWAP) {
        // lanes l < 32 (even half) take the odd half's values e < E/2 from lane l + 32,
        // which takes the even half's values e >= E/2: each lane then holds the sums
        // for its own store slots
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            cpx a = v[e], b = v[e + E / 2];
            swap_halves(a, b);
            if (ok) stg<(NT & 2) != 0>(base + t + G * (h * (E / 2) + e), cadd(a, b));
        }
        lds_sync<FW>();
    } else {
        lds_sync<FW>();
#pragma unroll
        for (int e = 0; e < E; ++e) area[lds_slot<FZ>(t + G * e)] = v[e];
        lds_sync<CW>();
        if (ok) {
            const cpx* a0 = lds + (pl * 2) * A;
            const cpx* a1 = a0 + A;
#pragma unroll
            for (int ee = 0; ee < E / 2; ++ee) {
                const int j = t + G * (h * (E / 2) + ee);
                stg<(NT & 2) != 0>(base + j, cadd(a0[lds_slot<FZ>(j)], a1[lds_slot<FZ>(j)]));
            }
        }
        lds_sync<CW>();
    }
}

// fused_body for the plans that pack pencils 0 and NX into one (fused_pack; 2D, so the plain
// spectrum): the same steps, with the packed pencil split into its two spectra between the
// transforms.  Every pencil of the block passes the same barriers; only the packed one
// exchanges its values through the LDS.
template <int N, int DIM, int MODE, int NT = NT_P3, bool EN = false, int RV = 0>
__device__ __forceinline__ void fused_body_pack(gp<cpx> __restrict__ X, gp<const cpx> __restrict__ tw, int pencil,
                                                int kx0, bool ok, int t, int h, int pl,
                                                cpx (&v)[GeoZ<N, RV>::EZ], const double (&sv)[GeoZ<N, RV>::EZ],
                                                cpx* lds, cpx* area, int NX, int NY, gp<double> part,
                                                bool packed, gp<const double> srow_n) {
    using Gm = GeoZ<N, RV>;
    using FZ = typename Gm::FZ;
    constexpr int E = Gm::EZ, G = Gm::GZ, A = Gm::AZ;
    constexpr bool FW = (G <= 64), CW = (2 * G <= 64);
    static_assert(DIM == 2 && MODE == SPEC_PLAIN, "pencils are packed in 2D only");
    if (h) twist_const<FZ, false>(v);
    fft<FZ, false, FW>(v, t, area, t, area, tw, h);
    double acc = 0.0, accn = 0.0;
    lds_sync<FW>();
    if (packed) {
#pragma unroll
        for (int e = 0; e < E; ++e) area[lds_slot<FZ>(t + G * e)] = v[e];
    }
    lds_sync<FW>();
    if (packed) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = t + G * e, m = 2 * j + h;
            const int jm = h ? (N - 1 - j) : (j == 0 ? 0 : N - j);    // the half index of -m
            const cpx w = area[lds_slot<FZ>(jm)];
            const cpx a = cmk(0.5 * (v[e].x + w.x), 0.5 * (v[e].y - w.y));   // A = (C + conj W) / 2
            const cpx b = cmk(0.5 * (v[e].x - w.x), 0.5 * (v[e].y + w.y));   // i B = (C - conj W) / 2
            const double sn = ldg<(NT & 4) != 0>(srow_n + (m <= N ? m : 2 * N - m));
            if constexpr (EN) {
                acc += sv[e] * (a.x * a.x + a.y * a.y);
                accn += sn * (b.x * b.x + b.y * b.y);
            }
            v[e] = cadd(cscale(a, sv[e]), cscale(b, sn));
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (EN) acc += sv[e] * (v[e].x * v[e].x + v[e].y * v[e].y);
            v[e] = cscale(v[e], sv[e]);
        }
    }
    if constexpr (EN) {
        fused_energy_store<N, DIM, RV>(acc, ok, pencil, kx0, t, h, pl, NX, NY, part);
        fused_energy_store<N, DIM, RV>(accn, packed, NX, kx0, t, h, pl, NX, NY, part);
    }
    lds_sync<FW>();
    fft_t<FZ, true, FW>(v, t, area, t, area, tw, h);
    gp<cpx> base = X + (size_t)pencil * N;
    gp<cpx> base_n = X + (size_t)NX * N;
    // the packed pencil stores its real part to pencil 0 and its imaginary part to pencil NX
    auto store = [&](int j, cpx r) {
        if (packed) {
            stg<(NT & 2) != 0>(base + j, cmk(r.x, 0.0));
            stg<(NT & 2) != 0>(base_n + j, cmk(r.y, 0.0));
        } else {
            stg<(NT & 2) != 0>(base + j, r);
        }
    };
    if constexpr (FusedRoles<N, RV>::SWAP) {
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            cpx a = v[e], b = v[e + E / 2];
            swap_halves(a, b);
            if (ok) store(t + G * (h * (E / 2) + e), cadd(a, b));
        }
        lds_sync<FW>();
    } else {
        lds_sync<FW>();
#pragma unroll
        for (int e = 0; e < E; ++e) area[lds_slot<FZ>(t + G * e)] = v[e];
        lds_sync<CW>();
        if (ok) {
            const cpx* a0 = lds + (pl * 2) * A;
            const cpx* a1 = a0 + A;
#pragma unroll
            for (int ee = 0; ee < E / 2; ++ee) {
                const int j = t + G * (h * (E / 2) + ee);
                store(j, cadd(a0[lds_slot<FZ>(j)], a1[lds_slot<FZ>(j)]));
            }
        }
        lds_sync<CW>();
    }
}

// One pencil group of the fused pass without prefetch (the batched launches).
// PZ: pencils per block (a tile-shape variant: the same bits for every PZ); RV: radix plan
// (FusedPlan)
template <int N, int DIM, int MODE, int NT = NT_P3, bool CUBE = true, int PZ = Geo<N>::PPZ, bool EN = false,
          int RV = 0>
__device__ __forceinline__ void fused_group(gp<cpx> __restrict__ X, gp<const double> __restrict__ spec,
                                            gp<const cpx> __restrict__ tw, int npencils, int kx0,
                                            const DipoleArgs& dip, int g, int tid, bool active, cpx* lds,
                                            Ext ext = Ext(), gp<double> part = nullptr) {
    using Gm = GeoZ<N, RV>;
    constexpr int E = Gm::EZ, G = Gm::GZ, PP = PZ, A = Gm::AZ;
    const int NX = CUBE ? N : ext.nx, NY = CUBE ? N : ext.ny;
    int t, h, pl;
    FusedRoles<N, RV>::get(tid, t, h, pl);
    cpx* area = lds + (pl * 2 + h) * A;
    const int slot = g * PP + pl;
    // in 3D the pencil count is a multiple of 2n, so groups of PP pencils never run past it
    // when PP divides 2n; 2D has n + 1 pencils (n slots when pencils 0 and n ride together)
    constexpr bool FULL = CUBE && (DIM == 3 && (2 * N) % PP == 0);
    const bool ok = active && (FULL || slot < fused_slots<N, DIM, RV>(npencils));
    const int pencil = ok ? fused_pencil<N, DIM>(slot, NY) : 0;
    cpx v[E];
    double sv[E];
    if constexpr (fused_pack<N, DIM, RV>()) {
        const bool packed = ok && slot == 0;
        if (packed) fused_load_pair<N, NT, RV>(X, NX, t, v);
        else fused_load<N, DIM, NT, RV>(X, pencil, ok, t, v);
        fused_spec<N, DIM, NT, RV>(spec, pencil, kx0, ok, t, h, sv, NY);
        fused_body_pack<N, DIM, MODE, NT, EN, RV>(X, tw, pencil, kx0, ok, t, h, pl, v, sv, lds, area, NX, NY, part,
                                                  packed, fused_row<N, DIM>(spec, NX, kx0, NY));
    } else {
        fused_load<N, DIM, NT, RV>(X, pencil, ok, t, v);
        fused_spec<N, DIM, NT, RV>(spec, pencil, kx0, ok, t, h, sv, NY);
        fused_body<N, DIM, MODE, NT, EN, RV>(X, tw, pencil, kx0, ok, dip, t, h, pl, v, sv, lds, area, NX, NY, part);
    }
}

// EN: also the energy sum of every pencil into part (fused_energy_store); RV: radix plan.
template <int N, int DIM, int MODE, int NT = NT_P3, int PZ = Geo<N>::PPZ, bool EN = false, int RV = 0>
__global__ void __launch_bounds__((PZ * 2 * GeoZ<N, RV>::GZ)) k_fused(cpx* __restrict__ Xg, const double* __restrict__ specg,
                                                              const cpx* __restrict__ twg, int npencils, int kx0,
                                                              DipoleArgs dip, double* __restrict__ part = nullptr) {
    __shared__ cpx lds[PZ * 2 * GeoZ<N, RV>::AZ];
    const int ngroups = (fused_slots<N, DIM, RV>(npencils) + PZ - 1) / PZ;
    if constexpr (!gs_fused_persistent(DIM, N)) {
        // one pencil group per block (the grid must cover all groups).  Without the
        // persistent loop the compiler does not keep the stage twiddles of every thread
        // live across groups: at n = 2048 in 2D, 250 VGPRs instead of 256 + 154 accumulator
        // registers, two waves per SIMD instead of one
        if ((int)blockIdx.x < ngroups)
            fused_group<N, DIM, MODE, NT, true, PZ, EN, RV>((gp<cpx>)Xg, (gp<const double>)specg, (gp<const cpx>)twg,
                                                            npencils, kx0, dip, blockIdx.x, threadIdx.x, true, lds,
                                                            Ext(), (gp<double>)part);
    } else {
        for (int g = blockIdx.x; g < ngroups; g += gridDim.x)
            fused_group<N, DIM, MODE, NT, true, PZ, EN, RV>((gp<cpx>)Xg, (gp<const double>)specg, (gp<const cpx>)twg,
                                                            npencils, kx0, dip, g, threadIdx.x, true, lds, Ext(),
                                                            (gp<double>)part);
    }
}

// ---------------------------------------------------------------------------
// The passes on grids whose axes have their own n (Section 2.5 with per-axis n_j): the
// transform length N is the n of the axis the pass transforms, the other extents come in
// `ext`, and every row and pencil is bounds-checked.  One block per tile or pencil group.
// ---------------------------------------------------------------------------
template <int N, int NT>
__global__ void __launch_bounds__(Geo<N>::TX) k_x_r2c_g(const double* __restrict__ rho, cpx* __restrict__ X1,
                                                        const cpx* __restrict__ tw, Ext ext) {
    __shared__ cpx lds[Geo<N>::PPX * Geo<N>::A];
    x_r2c_tile<N, NT, false>((gp<const double>)rho, (gp<cpx>)X1, (gp<const cpx>)tw, blockIdx.x, blockIdx.y,
                             threadIdx.x, true, lds, ext);
}

template <int N, int NT, bool SC>
__global__ void __launch_bounds__(Geo<N>::TX) k_x_c2r_g(const cpx* __restrict__ X1, double* u,
                                                        const cpx* __restrict__ tw, Ext ext, double oscale) {
    __shared__ cpx lds[Geo<N>::PPX * Geo<N>::A];
    x_c2r_tile<N, NT, SC, false>((gp<const cpx>)X1, (gp<double>)u, (gp<const cpx>)tw, blockIdx.x, blockIdx.y,
                                 threadIdx.x, true, lds, ext, oscale);
}

template <int N, int NT>
__global__ void __launch_bounds__(Geo<N>::TY) k_y_fwd_g(const cpx* __restrict__ X1, cpx* __restrict__ X2,
                                                        const cpx* __restrict__ tw, int kx0, Ext ext) {
    __shared__ cpx lds[Geo<N>::PPY * Geo<N>::A];
    y_fwd_tile<N, NT, false>((gp<const cpx>)X1, (gp<cpx>)X2, (gp<const cpx>)tw, kx0, blockIdx.x, blockIdx.y,
                             threadIdx.x, true, lds, ext);
}

template <int N, int NT>
__global__ void __launch_bounds__(Geo<N>::TY) k_y_inv_g(const cpx* __restrict__ X2, cpx* __restrict__ X1,
                                                        const cpx* __restrict__ tw, int kx0, Ext ext) {
    __shared__ cpx lds[Geo<N>::PPY * Geo<N>::A];
    y_inv_tile<N, NT, false>((gp<const cpx>)X2, (gp<cpx>)X1, (gp<const cpx>)tw, kx0, blockIdx.x, blockIdx.y,
                             threadIdx.x, true, lds, ext);
}

template <int N, int DIM, int MODE, int NT, bool EN = false>
__global__ void __launch_bounds__(Geo<N>::TZ) k_fused_g(cpx* __restrict__ Xg, const double* __restrict__ specg,
                                                        const cpx* __restrict__ twg, int npencils, int kx0,
                                                        DipoleArgs dip, Ext ext, double* __restrict__ part = nullptr) {
    __shared__ cpx lds[Geo<N>::PPZ * 2 * Geo<N>::AZ];
    const int ngroups = (fused_slots<N, DIM>(npencils) + Geo<N>::PPZ - 1) / Geo<N>::PPZ;
    if ((int)blockIdx.x < ngroups)
        fused_group<N, DIM, MODE, NT, false, Geo<N>::PPZ, EN>((gp<cpx>)Xg, (gp<const double>)specg,
                                                              (gp<const cpx>)twg, npencils, kx0, dip, blockIdx.x,
                                                              threadIdx.x, true, lds, ext, (gp<double>)part);
}

}  // namespace gsk
