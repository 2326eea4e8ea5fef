// fft_core.hpp -- FP64 complex FFT building blocks for gfx950 (CDNA4).
//
// Every padded transform of the method (zero padding n -> 2n, cropping 2n -> n;
// Section 2.2 and the Remark on padding to [-2L, 2L]) is split into two
// length-n FFTs: the even outputs X[2k] are the FFT of x, the odd outputs
// X[2k+1] the FFT of x_j * exp(-i pi j/n).  This file provides the length-n
// engine those passes share.
//
// Engine layout: a transform of length N is carried by G = N/E threads, each
// holding E complex values in registers.  Before every stage a thread t holds
// elements t + G*e (e = 0..E-1).  A stage of radix R does E/R butterflies per
// thread (Stockham autosort, decimation in time: twiddle, then an in-register
// DFT_R), and the outputs are exchanged through LDS.  After the last stage the
// thread holds X[t + G*e] in natural order.  The thread that runs the first
// stage may differ from the one that runs the later ones (t1/lds1 versus
// t2/lds2): passes use that to turn a coalesced load of one layout into a
// coalesced store of another through the LDS exchange the FFT needs anyway.
//
// Twiddles come from a per-size table W[m] = exp(-i pi m / N), m < 2N,
// computed on the host in extended precision.
#pragma once

#include <hip/hip_runtime.h>

namespace gsk {

typedef double2 cpx;

__device__ __forceinline__ cpx cmk(double a, double b) { return make_double2(a, b); }
__device__ __forceinline__ cpx cadd(cpx a, cpx b) { return cmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cpx csub(cpx a, cpx b) { return cmk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cpx cscale(cpx a, double s) { return cmk(a.x * s, a.y * s); }
__device__ __forceinline__ cpx cmul(cpx a, cpx b) {
    return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ cpx cmulc(cpx a, cpx b) {
    return cmk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ cpx cconj(cpx a) { return cmk(a.x, -a.y); }
// a * (-i) for the forward sign, a * (+i) for the inverse one
template <bool INV> __device__ __forceinline__ cpx mul_mi(cpx a) {
    return INV ? cmk(-a.y, a.x) : cmk(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Exact unit roots exp(-2 pi i e / R) for R dividing 48 (radices 2,3,4,6,8,12,16).
// ---------------------------------------------------------------------------
struct CS { double c, s; };

// cos and sin of a*pi/24 for a = 0..12 (only multiples of 3 or 4 occur)
constexpr CS first_quadrant(int a) {
    return a == 0  ? CS{1.0, 0.0}
         : a == 3  ? CS{0.92387953251128675613, 0.38268343236508977173}
         : a == 4  ? CS{0.86602540378443864676, 0.5}
         : a == 6  ? CS{0.70710678118654752440, 0.70710678118654752440}
         : a == 8  ? CS{0.5, 0.86602540378443864676}
         : a == 9  ? CS{0.38268343236508977173, 0.92387953251128675613}
         : a == 12 ? CS{0.0, 1.0}
                   : CS{2.0, 2.0};   // unreachable for the supported radices
}

// cos/sin of 2 pi e / R
constexpr CS unit_root(int e, int R) {
    int a = ((e % R + R) % R) * (48 / R);     // angle = a * pi / 24, a in [0, 48)
    int q = a / 12, r = a % 12;
    CS b = first_quadrant(r);
    return q == 0 ? CS{b.c, b.s} : q == 1 ? CS{-b.s, b.c} : q == 2 ? CS{-b.c, -b.s} : CS{b.s, -b.c};
}

// x * W_R^e with W_R = exp(-2 pi i / R) (forward) or its conjugate (inverse)
template <int E, int R, bool INV> __device__ __forceinline__ cpx twiddle_const(cpx x) {
    constexpr int e = ((E % R) + R) % R;
    if constexpr (e == 0) {
        return x;
    } else if constexpr ((4 * e) % R == 0) {
        constexpr int quarter = (4 * e) / R;           // W = (-i)^quarter (forward)
        if constexpr (quarter == 1) return mul_mi<INV>(x);
        else if constexpr (quarter == 2) return cmk(-x.x, -x.y);
        else return mul_mi<!INV>(x);
    } else {
        constexpr CS w = unit_root(e, R);
        // forward: exp(-i theta) = c - i s; inverse: c + i s
        constexpr double s = INV ? w.s : -w.s;
        return cmk(x.x * w.c - x.y * s, x.x * s + x.y * w.c);
    }
}

// ---------------------------------------------------------------------------
// In-register DFTs on v[0], v[S], ..., v[(R-1) S] (S a compile-time stride).
// ---------------------------------------------------------------------------
template <int R, int S, bool INV> struct Dft;

template <int S, bool INV> struct Dft<2, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) {
        cpx a = v[0], b = v[S];
        v[0] = cadd(a, b);
        v[S] = csub(a, b);
    }
};

template <int S, bool INV> struct Dft<3, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) {
        constexpr double h = 0.86602540378443864676;   // sin(2 pi/3)
        cpx a = v[0], b = v[S], c = v[2 * S];
        cpx t = cadd(b, c);
        cpx m = cmk(a.x - 0.5 * t.x, a.y - 0.5 * t.y);
        cpx dd = csub(b, c);
        cpx d = INV ? cmk(-h * dd.y, h * dd.x) : cmk(h * dd.y, -h * dd.x);
        v[0] = cadd(a, t);
        v[S] = cadd(m, d);
        v[2 * S] = csub(m, d);
    }
};

template <int S, bool INV> struct Dft<4, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) {
        cpx a = v[0], b = v[S], c = v[2 * S], d = v[3 * S];
        cpx t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d);
        cpx t3 = mul_mi<INV>(csub(b, d));
        v[0] = cadd(t0, t2);
        v[2 * S] = csub(t0, t2);
        v[S] = cadd(t1, t3);
        v[3 * S] = csub(t1, t3);
    }
};

// DFT of length R1*R2 by one Cooley-Tukey split: j = R2 j1 + j2, k = k1 + R1 k2.
template <int R1, int R2, int S, bool INV> struct DftComposite {
    static constexpr int R = R1 * R2;
    template <int J2> __device__ __forceinline__ static void first(cpx* v) {
        Dft<R1, R2 * S, INV>::run(v + J2 * S);
    }
    __device__ __forceinline__ static void run(cpx* v) {
        // DFT_R1 over j1 for every j2; result A[j2][k1] at position R2 k1 + j2
        [&]<int... J>(std::integer_sequence<int, J...>) { (first<J>(v), ...); }
        (std::make_integer_sequence<int, R2>{});
        // twiddles W_R^{j2 k1}
        [&]<int... I>(std::integer_sequence<int, I...>) {
            ((v[((I / R2) * R2 + (I % R2)) * S] =
                  twiddle_const<(I % R2) * (I / R2), R, INV>(v[((I / R2) * R2 + (I % R2)) * S])), ...);
        }(std::make_integer_sequence<int, R>{});
        // DFT_R2 over j2 for every k1; X[k1 + R1 k2] lands at position R2 k1 + k2
        [&]<int... K>(std::integer_sequence<int, K...>) { (Dft<R2, S, INV>::run(v + R2 * K * S), ...); }
        (std::make_integer_sequence<int, R1>{});
        // register renaming into natural order
        cpx tmp[R];
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) tmp[k1 + R1 * k2] = v[(R2 * k1 + k2) * S];
#pragma unroll
        for (int k = 0; k < R; ++k) v[k * S] = tmp[k];
    }
};

template <int S, bool INV> struct Dft<6, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) { DftComposite<2, 3, S, INV>::run(v); }
};
template <int S, bool INV> struct Dft<8, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) { DftComposite<2, 4, S, INV>::run(v); }
};
template <int S, bool INV> struct Dft<12, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) { DftComposite<4, 3, S, INV>::run(v); }
};
template <int S, bool INV> struct Dft<16, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) { DftComposite<4, 4, S, INV>::run(v); }
};

// ---------------------------------------------------------------------------
// Per-size plans: E values per thread and the stage radices (product = N).
// ---------------------------------------------------------------------------
template <int N> struct FftCfg;
#define GSK_FFT_CFG(N_, E_, NS_, R0_, R1_, R2_, R3_)                              \
    template <> struct FftCfg<N_> {                                               \
        static constexpr int E = E_, NS = NS_, G = N_ / E_;                       \
        static constexpr int R[4] = {R0_, R1_, R2_, R3_};                         \
    };
GSK_FFT_CFG(8, 8, 1, 8, 1, 1, 1)
GSK_FFT_CFG(12, 12, 2, 4, 3, 1, 1)
GSK_FFT_CFG(16, 16, 1, 16, 1, 1, 1)
GSK_FFT_CFG(24, 24, 2, 8, 3, 1, 1)
GSK_FFT_CFG(32, 8, 2, 4, 8, 1, 1)
GSK_FFT_CFG(48, 12, 3, 4, 4, 3, 1)
GSK_FFT_CFG(64, 8, 2, 8, 8, 1, 1)
GSK_FFT_CFG(96, 12, 4, 4, 4, 2, 3)
GSK_FFT_CFG(128, 16, 2, 16, 8, 1, 1)
GSK_FFT_CFG(192, 12, 4, 4, 4, 4, 3)
GSK_FFT_CFG(256, 16, 2, 16, 16, 1, 1)
GSK_FFT_CFG(512, 8, 3, 8, 8, 8, 1)
GSK_FFT_CFG(1024, 16, 3, 16, 16, 4, 1)
GSK_FFT_CFG(2048, 16, 3, 16, 16, 8, 1)
#undef GSK_FFT_CFG

// LDS area of one transform: one 16-byte pad slot after every 16 elements so that
// the strided Stockham scatters spread over the banks.
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }
template <int N> struct LdsArea { static constexpr int size = N + N / 16 + 1; };

// One Stockham stage on registers: twiddles (unless first) and E/R DFTs of radix R.
template <int N, int E, int R, int NSPRE, bool INV>
__device__ __forceinline__ void stage_compute(cpx (&v)[E], int t, const cpx* __restrict__ tw) {
    constexpr int G = N / E, B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        if constexpr (NSPRE > 1) {
            const int j = t + b * G;
            const int base = (j % NSPRE) * (N / (NSPRE * R));
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cpx w = tw[2 * base * r];     // W_N^{base r} = W_{2N}^{2 base r}
                v[b + r * B] = INV ? cmulc(v[b + r * B], w) : cmul(v[b + r * B], w);
            }
        }
        Dft<R, B, INV>::run(&v[b]);
    }
}

template <int N, int E, int R, int NSPRE>
__device__ __forceinline__ void stage_scatter(const cpx (&v)[E], int t, cpx* lds) {
    constexpr int G = N / E, B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + b * G;
        const int base = (j / NSPRE) * NSPRE * R + (j % NSPRE);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lds_pad(base + r * NSPRE)] = v[b + r * B];
    }
}

template <int N, int E>
__device__ __forceinline__ void stage_gather(cpx (&v)[E], int t, const cpx* lds) {
    constexpr int G = N / E;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = lds[lds_pad(t + G * e)];
}

// Full length-N transform.  On entry thread t1 holds x[t1 + G e]; on exit thread t2
// holds X[t2 + G e].  lds1/lds2 are the LDS areas of the transform as seen by the
// two thread roles.  Contains block barriers: every thread of the block must call
// it, and the areas must not be in use by other threads when it is entered.
template <int N, bool INV>
__device__ __forceinline__ void fft(cpx (&v)[FftCfg<N>::E], int t1, cpx* lds1, int t2, cpx* lds2,
                                    const cpx* __restrict__ tw) {
    using C = FftCfg<N>;
    constexpr int E = C::E;
    constexpr int R0 = C::R[0], R1 = C::R[1], R2 = C::R[2], R3 = C::R[3];
    stage_compute<N, E, R0, 1, INV>(v, t1, tw);
    if constexpr (C::NS >= 2) {
        stage_scatter<N, E, R0, 1>(v, t1, lds1);
        __syncthreads();
        stage_gather<N, E>(v, t2, lds2);
        stage_compute<N, E, R1, R0, INV>(v, t2, tw);
    }
    if constexpr (C::NS >= 3) {
        __syncthreads();
        stage_scatter<N, E, R1, R0>(v, t2, lds2);
        __syncthreads();
        stage_gather<N, E>(v, t2, lds2);
        stage_compute<N, E, R2, R0 * R1, INV>(v, t2, tw);
    }
    if constexpr (C::NS >= 4) {
        __syncthreads();
        stage_scatter<N, E, R2, R0 * R1>(v, t2, lds2);
        __syncthreads();
        stage_gather<N, E>(v, t2, lds2);
        stage_compute<N, E, R3, R0 * R1 * R2, INV>(v, t2, tw);
    }
}

}  // namespace gsk
