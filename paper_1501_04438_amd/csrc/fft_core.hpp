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
// The odd half's twist x_j exp(-i pi j/n) can ride through the stages (fft with h = 1),
// and an inverse followed by the cropping twist runs on the transposed engine (fft_t).
//
// Twiddles come from a per-size table W[m] = exp(-i pi m / N), m < 2N,
// computed on the host in extended precision.
#pragma once

#include <hip/hip_runtime.h>

namespace gsk {

// Global-memory pointer.  Device functions take global data through this type so
// that every access compiles to a global (not flat) instruction, also where the
// pointer was read from memory rather than passed as a kernel argument.
template <class T> using gp = __attribute__((address_space(1))) T*;

// complex FP64 as a native two-lane vector: copies from any address space are
// plain loads and stores
typedef double cpx __attribute__((ext_vector_type(2)));

__device__ __forceinline__ cpx cmk(double a, double b) {
    cpx r = {a, b};
    return r;
}
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
// Unit roots exp(-2 pi i e / R), correctly rounded, for R dividing 96 (radices
// 2,3,4,6,8,12,16 and the padding twists of 16, 24, 32 and 48 points), 40 (radices 5
// and 10, the twists of 20 points) or 56 (radices 7 and 14, the twists of 28 points).
// ---------------------------------------------------------------------------
struct CS { double c, s; };

// cos and sin of a*pi/48 for the a in [0, 24] that occur
constexpr CS first_quadrant(int a) {
    return a == 0  ? CS{1.0, 0.0}
         : a == 2  ? CS{0.991444861373810411145, 0.130526192220051591548}
         : a == 3  ? CS{0.980785280403230449126, 0.195090322016128267848}
         : a == 4  ? CS{0.96592582628906828675, 0.258819045102520762349}
         : a == 6  ? CS{0.923879532511286756128, 0.382683432365089771728}
         : a == 8  ? CS{0.866025403784438646764, 0.5}
         : a == 9  ? CS{0.831469612302545237079, 0.555570233019602224743}
         : a == 10 ? CS{0.79335334029123516458, 0.608761429008720639416}
         : a == 12 ? CS{0.707106781186547524401, 0.707106781186547524401}
         : a == 14 ? CS{0.608761429008720639416, 0.79335334029123516458}
         : a == 15 ? CS{0.555570233019602224743, 0.831469612302545237079}
         : a == 16 ? CS{0.5, 0.866025403784438646764}
         : a == 18 ? CS{0.382683432365089771728, 0.923879532511286756128}
         : a == 20 ? CS{0.258819045102520762349, 0.96592582628906828675}
         : a == 21 ? CS{0.195090322016128267848, 0.980785280403230449126}
         : a == 22 ? CS{0.130526192220051591548, 0.991444861373810411145}
         : a == 24 ? CS{0.0, 1.0}
                   : CS{2.0, 2.0};   // unreachable for the supported radices
}

// cos and sin of a*pi/20, a in [0, 10]
constexpr CS first_quadrant20(int a) {
    return a == 0  ? CS{1.0, 0.0}
         : a == 1  ? CS{0.98768834059513772619, 0.15643446504023086901}
         : a == 2  ? CS{0.951056516295153572116, 0.309016994374947424102}
         : a == 3  ? CS{0.89100652418836786236, 0.45399049973954679156}
         : a == 4  ? CS{0.809016994374947424102, 0.587785252292473129169}
         : a == 5  ? CS{0.707106781186547524401, 0.707106781186547524401}
         : a == 6  ? CS{0.587785252292473129169, 0.809016994374947424102}
         : a == 7  ? CS{0.45399049973954679156, 0.89100652418836786236}
         : a == 8  ? CS{0.309016994374947424102, 0.951056516295153572116}
         : a == 9  ? CS{0.15643446504023086901, 0.98768834059513772619}
         : a == 10 ? CS{0.0, 1.0}
                   : CS{2.0, 2.0};
}

// cos and sin of a*pi/28, a in [0, 14]
constexpr CS first_quadrant28(int a) {
    return a == 0  ? CS{1.0, 0.0}
         : a == 1  ? CS{0.993712209893242583533, 0.111964476103307858469}
         : a == 2  ? CS{0.974927912181823607018, 0.222520933956314404289}
         : a == 3  ? CS{0.943883330308367562895, 0.330279061955167081775}
         : a == 4  ? CS{0.900968867902419126236, 0.433883739117558120476}
         : a == 5  ? CS{0.846724199228284168353, 0.532032076515336563558}
         : a == 6  ? CS{0.781831482468029808708, 0.623489801858733530525}
         : a == 7  ? CS{0.707106781186547524401, 0.707106781186547524401}
         : a == 8  ? CS{0.623489801858733530525, 0.781831482468029808708}
         : a == 9  ? CS{0.532032076515336563558, 0.846724199228284168353}
         : a == 10 ? CS{0.433883739117558120476, 0.900968867902419126236}
         : a == 11 ? CS{0.330279061955167081775, 0.943883330308367562895}
         : a == 12 ? CS{0.222520933956314404289, 0.974927912181823607018}
         : a == 13 ? CS{0.111964476103307858469, 0.993712209893242583533}
         : a == 14 ? CS{0.0, 1.0}
                   : CS{2.0, 2.0};
}

// Angle unit pi / B of the table that holds the roots of order R (0: none)
constexpr int root_base(int R) { return 96 % R == 0 ? 48 : 40 % R == 0 ? 20 : 56 % R == 0 ? 28 : 0; }

// cos/sin of 2 pi e / R
constexpr CS unit_root(int e, int R) {
    const int B = root_base(R), Q = B / 2;
    int a = ((e % R + R) % R) * (2 * B / R);  // angle = a * pi / B, a in [0, 2B)
    int q = a / Q, r = a % Q;
    CS b = B == 48 ? first_quadrant(r) : B == 20 ? first_quadrant20(r) : first_quadrant28(r);
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
        static_assert(root_base(R) != 0, "unit roots of this order are not tabulated");
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

// Five points: X_k = x0 + sum_j x_j W^{jk}.  With t1 = x1 + x4, t2 = x2 + x3, t3 = x1 - x4,
// t4 = x2 - x3 and c_m, s_m the cosine and sine of 2 pi m / 5:
//   X1, X4 = x0 + c1 t1 + c2 t2 -+ i (s1 t3 + s2 t4)
//   X2, X3 = x0 + c2 t1 + c1 t2 -+ i (s2 t3 - s1 t4)      (forward; signs of i swapped inverse)
template <int S, bool INV> struct Dft<5, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) {
        constexpr double c1 = 0.309016994374947424102, s1 = 0.951056516295153572116;
        constexpr double c2 = -0.809016994374947424102, s2 = 0.587785252292473129169;
        const cpx x0 = v[0];
        const cpx t1 = cadd(v[S], v[4 * S]), t3 = csub(v[S], v[4 * S]);
        const cpx t2 = cadd(v[2 * S], v[3 * S]), t4 = csub(v[2 * S], v[3 * S]);
        const cpx a1 = cmk(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
        const cpx a2 = cmk(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
        const cpx b1 = mul_mi<INV>(cmk(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
        const cpx b2 = mul_mi<INV>(cmk(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
        v[0] = cadd(x0, cadd(t1, t2));
        v[S] = cadd(a1, b1);
        v[4 * S] = csub(a1, b1);
        v[2 * S] = cadd(a2, b2);
        v[3 * S] = csub(a2, b2);
    }
};

// Seven points, the same pairing: t_m = x_m + x_{7-m}, d_m = x_m - x_{7-m} (m = 1, 2, 3),
//   X_k, X_{7-k} = x0 + sum_m cos(2 pi m k / 7) t_m -+ i sum_m sin(2 pi m k / 7) d_m.
template <int S, bool INV> struct Dft<7, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) {
        constexpr double c1 = 0.623489801858733530525, s1 = 0.781831482468029808708;
        constexpr double c2 = -0.222520933956314404289, s2 = 0.974927912181823607018;
        constexpr double c3 = -0.900968867902419126236, s3 = 0.433883739117558120476;
        const cpx x0 = v[0];
        const cpx t1 = cadd(v[S], v[6 * S]), d1 = csub(v[S], v[6 * S]);
        const cpx t2 = cadd(v[2 * S], v[5 * S]), d2 = csub(v[2 * S], v[5 * S]);
        const cpx t3 = cadd(v[3 * S], v[4 * S]), d3 = csub(v[3 * S], v[4 * S]);
        // cos(2 pi m k / 7) and sin(2 pi m k / 7) for k = 1, 2, 3 (mk reduced mod 7)
        const cpx a1 = cmk(x0.x + c1 * t1.x + c2 * t2.x + c3 * t3.x, x0.y + c1 * t1.y + c2 * t2.y + c3 * t3.y);
        const cpx a2 = cmk(x0.x + c2 * t1.x + c3 * t2.x + c1 * t3.x, x0.y + c2 * t1.y + c3 * t2.y + c1 * t3.y);
        const cpx a3 = cmk(x0.x + c3 * t1.x + c1 * t2.x + c2 * t3.x, x0.y + c3 * t1.y + c1 * t2.y + c2 * t3.y);
        const cpx b1 = mul_mi<INV>(cmk(s1 * d1.x + s2 * d2.x + s3 * d3.x, s1 * d1.y + s2 * d2.y + s3 * d3.y));
        const cpx b2 = mul_mi<INV>(cmk(s2 * d1.x - s3 * d2.x - s1 * d3.x, s2 * d1.y - s3 * d2.y - s1 * d3.y));
        const cpx b3 = mul_mi<INV>(cmk(s3 * d1.x - s1 * d2.x + s2 * d3.x, s3 * d1.y - s1 * d2.y + s2 * d3.y));
        v[0] = cadd(x0, cadd(t1, cadd(t2, t3)));
        v[S] = cadd(a1, b1);
        v[6 * S] = csub(a1, b1);
        v[2 * S] = cadd(a2, b2);
        v[5 * S] = csub(a2, b2);
        v[3 * S] = cadd(a3, b3);
        v[4 * S] = csub(a3, b3);
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
template <int S, bool INV> struct Dft<10, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) { DftComposite<2, 5, S, INV>::run(v); }
};
template <int S, bool INV> struct Dft<14, S, INV> {
    __device__ __forceinline__ static void run(cpx* v) { DftComposite<2, 7, S, INV>::run(v); }
};

// ---------------------------------------------------------------------------
// Transform plans: length N carried by G = N/E threads with E values each, the
// stage radices R[0..NS-1] (product N, each dividing E).  SLOTS selects the LDS
// layout of the exchanges (see lds_slot).
// ---------------------------------------------------------------------------
enum { SLOTS_PAD16 = 0, SLOTS_PAD8 = 1 };
template <int N_, int E_, int NS_, int R0_, int R1_ = 1, int R2_ = 1, int R3_ = 1, int SLOTS_ = SLOTS_PAD16>
struct FftPlan {
    static constexpr int N = N_, E = E_, NS = NS_, G = N_ / E_, SLOTS = SLOTS_;
    static constexpr int R[4] = {R0_, R1_, R2_, R3_};
};

// Default plans (few stages: one LDS exchange for n <= 256).
template <int N> struct FftCfg;
template <> struct FftCfg<8> : FftPlan<8, 8, 1, 8> {};
template <> struct FftCfg<12> : FftPlan<12, 12, 2, 4, 3> {};
template <> struct FftCfg<16> : FftPlan<16, 8, 2, 4, 4> {};
template <> struct FftCfg<24> : FftPlan<24, 12, 2, 4, 6> {};
template <> struct FftCfg<32> : FftPlan<32, 8, 2, 4, 8> {};
template <> struct FftCfg<48> : FftPlan<48, 12, 3, 4, 4, 3> {};
template <> struct FftCfg<64> : FftPlan<64, 8, 2, 8, 8> {};
template <> struct FftCfg<96> : FftPlan<96, 12, 4, 4, 4, 2, 3> {};
template <> struct FftCfg<128> : FftPlan<128, 8, 3, 8, 4, 4> {};
template <> struct FftCfg<192> : FftPlan<192, 12, 4, 4, 4, 4, 3> {};
template <> struct FftCfg<256> : FftPlan<256, 16, 2, 16, 16> {};
template <> struct FftCfg<512> : FftPlan<512, 8, 3, 8, 8, 8> {};
template <> struct FftCfg<1024> : FftPlan<1024, 16, 3, 16, 16, 4> {};
template <> struct FftCfg<2048> : FftPlan<2048, 16, 3, 16, 16, 8> {};
// 3 * 2^7 and up (the transform grids of padding to B_3 at n = 256, 512, 1024)
template <> struct FftCfg<384> : FftPlan<384, 12, 4, 4, 4, 4, 6> {};
template <> struct FftCfg<768> : FftPlan<768, 12, 4, 4, 4, 4, 12> {};
template <> struct FftCfg<1536> : FftPlan<1536, 24, 4, 8, 8, 8, 3> {};
// 5-smooth and 7-smooth lengths: 20 or 28 values per thread
template <> struct FftCfg<20> : FftPlan<20, 20, 2, 4, 5> {};
template <> struct FftCfg<40> : FftPlan<40, 20, 2, 4, 10> {};
template <> struct FftCfg<80> : FftPlan<80, 20, 3, 4, 4, 5> {};
template <> struct FftCfg<160> : FftPlan<160, 20, 3, 4, 4, 10> {};
template <> struct FftCfg<320> : FftPlan<320, 20, 4, 4, 4, 4, 5> {};
template <> struct FftCfg<640> : FftPlan<640, 20, 4, 4, 4, 4, 10> {};
template <> struct FftCfg<28> : FftPlan<28, 28, 2, 4, 7> {};
template <> struct FftCfg<56> : FftPlan<56, 28, 2, 4, 14> {};
template <> struct FftCfg<112> : FftPlan<112, 28, 3, 4, 4, 7> {};
template <> struct FftCfg<224> : FftPlan<224, 28, 3, 4, 4, 14> {};

// Plans for the fused spectrum pass, whose registers also hold the spectrum row:
// fewer values per thread where that matters (n = 256: 8 values, radices 8, 8, 4,
// a 32-thread transform, one LDS pad slot per 8 elements).
template <int N> struct FftCfgFused : FftCfg<N> {};
template <> struct FftCfgFused<256> : FftPlan<256, 8, 3, 8, 8, 4, 1, SLOTS_PAD8> {};
// n = 1024: 8 values per thread instead of 16 (no accumulator-register spills, two waves
// per SIMD instead of one); measured 30.0 -> 26.4 ms for the 1024^3 fused pass and
// 0.026 -> 0.024 ms for the 2D 1024^2 one.  The x and y passes keep the 16-value plan,
// which is faster for them.
template <> struct FftCfgFused<1024> : FftPlan<1024, 8, 4, 8, 8, 4, 4> {};

// Radix-plan variants of the fused pass that the plan autotuner times against the default
// (RV = 1; elsewhere RV = 1 names the default plan): the other value count per thread at the
// power-of-two lengths from 128 up (16 values where the default holds 8, and 8 where it holds
// 16), so the autotuner chooses between more registers per thread with fewer stages and
// exchanges, and more threads with more of them.  A different factorisation rounds
// differently: a plan on a variant agrees with the default to rounding, not bitwise.
// (RV = 0 names FftCfgFused<N> itself, so the default kernels are the same instances.)
template <int N, int RV> struct FusedPlanSel { using type = FftCfgFused<N>; };
template <> struct FusedPlanSel<128, 1> { using type = FftPlan<128, 16, 2, 16, 8>; };
template <> struct FusedPlanSel<256, 1> { using type = FftPlan<256, 16, 2, 16, 16>; };
template <> struct FusedPlanSel<512, 1> { using type = FftPlan<512, 16, 3, 16, 16, 2>; };
template <> struct FusedPlanSel<1024, 1> { using type = FftPlan<1024, 16, 3, 16, 16, 4>; };
template <> struct FusedPlanSel<2048, 1> { using type = FftPlan<2048, 8, 4, 8, 8, 4, 8>; };
template <int N, int RV> using FusedPlan = typename FusedPlanSel<N, RV>::type;
template <int N> constexpr bool fused_radix_variant() {
    return N == 128 || N == 256 || N == 512 || N == 1024 || N == 2048;
}

// The same for the x passes (XV = 1; the x-forward and x-inverse passes choose apart): the
// other value count per thread than FftCfg at the same lengths (XV = 0: FftCfg<N> itself).
template <int N, int XV> struct XPlanSel { using type = FftCfg<N>; };
template <> struct XPlanSel<128, 1> { using type = FftPlan<128, 16, 2, 16, 8>; };
template <> struct XPlanSel<256, 1> { using type = FftPlan<256, 8, 3, 8, 8, 4>; };
template <> struct XPlanSel<512, 1> { using type = FftPlan<512, 16, 3, 16, 16, 2>; };
template <> struct XPlanSel<1024, 1> { using type = FftPlan<1024, 8, 4, 8, 8, 4, 4>; };
template <> struct XPlanSel<2048, 1> { using type = FftPlan<2048, 8, 4, 8, 8, 4, 8>; };
template <int N, int XV> using XPlan = typename XPlanSel<N, XV>::type;
template <int N> constexpr bool x_radix_variant() { return fused_radix_variant<N>(); }

// Block barrier ordering LDS only: global loads in flight (prefetches) are not
// drained, unlike __syncthreads(), whose workgroup fence covers global memory.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS ordering among the lanes of one wave (LDS operations of a wave execute in
// order; this keeps the compiler from reordering across it).
__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <bool WAVE> __device__ __forceinline__ void lds_sync() {
    if constexpr (WAVE) lds_wave_sync();
    else lds_barrier();
}

// LDS area of one transform: one 16-byte pad slot after every 16 elements so that
// the strided Stockham scatters spread over the banks.
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }
template <int N> struct LdsArea { static constexpr int size = N + N / 16 + 1; };
// Slot of element i in the LDS area of a plan C (SLOTS_PAD8: one pad slot per 8).
// Bank rules measured on gfx950: a 16-byte LDS store serves 8 consecutive lanes per
// cycle, which must hit distinct slots mod 8 (128 bytes); a 16-byte LDS load serves
// 16 lanes per cycle (the lane sets of equal bit 5 and equal parity of bits 2-4),
// which must hit distinct slots mod 16 (256 bytes).  For the 8 x 8 x 4 plan of 256
// points (32-thread transforms, two per wave) the radix-8 scatter of the first
// stage is then conflict-free with PAD8 and takes two cycles per lane group with
// PAD16.  (A XOR swizzle removes the gather conflicts as well, but its addresses
// cost registers or instructions that the fused pass cannot spare: measured slower.)
template <class C> __host__ __device__ constexpr int lds_slot(int i) {
    if constexpr (C::SLOTS == SLOTS_PAD8) return i + (i >> 3);
    else return lds_pad(i);
}
template <class C> struct LdsAreaOf {
    static constexpr int size = (C::SLOTS == SLOTS_PAD8) ? C::N + C::N / 8 + 1 : LdsArea<C::N>::size;
};

// v[r S] *= w^r (conj for INV), r = 1..R-1, with w^{4a+c} = (w^4)^a w^c formed from
// w1 = w and w4 = w^4: at most three multiplications deep.
template <int R, int S, bool INV>
__device__ __forceinline__ void mul_powers(cpx* v, cpx w1, cpx w4) {
    const cpx p2 = cmul(w1, w1);
    const cpx p3 = cmul(p2, w1);
    const cpx q2 = cmul(w4, w4);
    const cpx q3 = cmul(q2, w4);
#pragma unroll
    for (int r = 1; r < R; ++r) {
        const int a = r / 4, c = r % 4;
        const cpx pc = c == 1 ? w1 : (c == 2 ? p2 : p3);
        const cpx qa = a == 1 ? w4 : (a == 2 ? q2 : q3);
        const cpx w = (a == 0) ? pc : (c == 0 ? qa : cmul(qa, pc));
        v[r * S] = INV ? cmulc(v[r * S], w) : cmul(v[r * S], w);
    }
}

// Twiddle roots of a stage (NSPRE > 1) for butterfly j: W_N^base = W_2N^{2 base} and its
// fourth power.  With h = 1 the root is W_2N^{2 base + N/(NSPRE R)}: the padding twist
// x_j W_2N^j of the odd half, carried through the stages (see fft).
template <int N, int R, int NSPRE>
__device__ __forceinline__ void stage_roots(int j, int h, gp<const cpx> __restrict__ tw, cpx& w1, cpx& w4) {
    constexpr int U = N / (NSPRE * R);
    const int base = (j % NSPRE) * U;
    w1 = tw[2 * base + h * U];
    w4 = (R > 4) ? tw[8 * base + 4 * h * U] : w1;          // 8 base + 4 U < 2N for R > 4
}

// One Stockham stage on registers: twiddles (unless first) and E/R DFTs of radix R.
// The twiddles W_N^{base r} are powers of W_N^{base} (two table reads per butterfly).
template <int N, int E, int R, int NSPRE, bool INV>
__device__ __forceinline__ void stage_compute(cpx (&v)[E], int t, gp<const cpx> __restrict__ tw, int h = 0) {
    constexpr int G = N / E, B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        if constexpr (NSPRE > 1) {
            cpx w1, w4;
            stage_roots<N, R, NSPRE>(t + b * G, h, tw, w1, w4);
            mul_powers<R, B, INV>(&v[b], w1, w4);
        }
        Dft<R, B, INV>::run(&v[b]);
    }
}

// The same stage transposed: the DFTs first, then the twiddles (for the transposed engine).
template <int N, int E, int R, int NSPRE, bool INV>
__device__ __forceinline__ void stage_compute_t(cpx (&v)[E], int t, gp<const cpx> __restrict__ tw, int h) {
    constexpr int G = N / E, B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        Dft<R, B, INV>::run(&v[b]);
        if constexpr (NSPRE > 1) {
            cpx w1, w4;
            stage_roots<N, R, NSPRE>(t + b * G, h, tw, w1, w4);
            mul_powers<R, B, INV>(&v[b], w1, w4);
        }
    }
}

// The constant part of the padding twist: v[b + r B] *= W_{2 R0}^r (conjugated when INV),
// r the input index within the first stage's radix-R0 butterflies.
template <class P, bool INV>
__device__ __forceinline__ void twist_const(cpx (&v)[P::E]) {
    constexpr int E = P::E, R0 = P::R[0], B = E / R0;
    [&]<int... I>(std::integer_sequence<int, I...>) {
        ((v[I] = twiddle_const<I / B, 2 * R0, INV>(v[I])), ...);
    }(std::make_integer_sequence<int, E>{});
}

// Padding twist before a forward transform, applied on its own: x[j] *= W_2N^j for
// j = t + G e, as W_2N^t (one table read) times the constant W_2E^e (for a pass whose
// registers do not leave room for the twisted roots of fft's h = 1).
template <class P>
__device__ __forceinline__ void twist_in(cpx (&v)[P::E], int t, gp<const cpx> __restrict__ tw) {
    constexpr int E = P::E;
    const cpx c = tw[t];
    [&]<int... I>(std::integer_sequence<int, I...>) {
        ((v[I] = cmul(twiddle_const<I, 2 * E, false>(v[I]), c)), ...);
    }(std::make_integer_sequence<int, E>{});
}

template <class C, int R, int NSPRE>
__device__ __forceinline__ void stage_scatter(const cpx (&v)[C::E], int t, cpx* lds) {
    constexpr int E = C::E, G = C::G, B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + b * G;
        const int base = (j / NSPRE) * NSPRE * R + (j % NSPRE);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lds_slot<C>(base + r * NSPRE)] = v[b + r * B];
    }
}

template <class C>
__device__ __forceinline__ void stage_gather(cpx (&v)[C::E], int t, const cpx* lds) {
    constexpr int E = C::E, G = C::G;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = lds[lds_slot<C>(t + G * e)];
}

// Full length-N transform.  On entry thread t1 holds x[t1 + G e]; on exit thread t2
// holds X[t2 + G e].  lds1/lds2 are the LDS areas of the transform as seen by the
// two thread roles.  WAVE = true when both roles coincide and the G threads of a
// transform lie in one wave (only wave-level ordering is then needed); otherwise
// it contains block barriers and every thread of the block must call it.  The
// areas must not be in use by other threads when it is entered.
//
// h = 1 (a per-thread value) computes the transform of x_j W_2N^j, the odd half of a padded
// transform, without a separate twist: writing j = (t + G b) + r N/R0 for input r of a
// first-stage butterfly, W_2N^j = W_2N^{t + G b} W_{2 R0}^r; the caller applies the constant
// W_{2 R0}^r (twist_const) and the factor W_2N^{t + G b}, common to the butterfly, rides on
// its outputs.  After a stage with NSPRE = P and radix R the factor at position q is
// W_2N^{floor(q / PR)}; at the next stage it becomes, for input r of a butterfly,
// W_2N^{floor(j / P)} W_2N^{r N / (P R)}: the second part joins that stage's twiddle root
// (stage_roots), the first again rides on the outputs, and after the last stage (PR = N) it is 1.
template <class C, bool INV, bool WAVE = false>
__device__ __forceinline__ void fft(cpx (&v)[C::E], int t1, cpx* lds1, int t2, cpx* lds2,
                                    gp<const cpx> __restrict__ tw, int h = 0) {
    constexpr int N = C::N;
    constexpr int E = C::E;
    constexpr int R0 = C::R[0], R1 = C::R[1], R2 = C::R[2], R3 = C::R[3];
    stage_compute<N, E, R0, 1, INV>(v, t1, tw);
    if constexpr (C::NS >= 2) {
        stage_scatter<C, R0, 1>(v, t1, lds1);
        lds_sync<WAVE>();
        stage_gather<C>(v, t2, lds2);
        stage_compute<N, E, R1, R0, INV>(v, t2, tw, h);
    }
    if constexpr (C::NS >= 3) {
        lds_sync<WAVE>();
        stage_scatter<C, R1, R0>(v, t2, lds2);
        lds_sync<WAVE>();
        stage_gather<C>(v, t2, lds2);
        stage_compute<N, E, R2, R0 * R1, INV>(v, t2, tw, h);
    }
    if constexpr (C::NS >= 4) {
        lds_sync<WAVE>();
        stage_scatter<C, R2, R0 * R1>(v, t2, lds2);
        lds_sync<WAVE>();
        stage_gather<C>(v, t2, lds2);
        stage_compute<N, E, R3, R0 * R1 * R2, INV>(v, t2, tw, h);
    }
}

// Reverse exchange of the stage (R, NSPRE): each thread writes its values where fft's
// gather reads them and reads them back where fft's scatter wrote them.
template <class C>
__device__ __forceinline__ void stage_ungather(const cpx (&v)[C::E], int t, cpx* lds) {
    constexpr int E = C::E, G = C::G;
#pragma unroll
    for (int e = 0; e < E; ++e) lds[lds_slot<C>(t + G * e)] = v[e];
}

template <class C, int R, int NSPRE>
__device__ __forceinline__ void stage_unscatter(cpx (&v)[C::E], int t, const cpx* lds) {
    constexpr int E = C::E, G = C::G, B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + b * G;
        const int base = (j / NSPRE) * NSPRE * R + (j % NSPRE);
#pragma unroll
        for (int r = 0; r < R; ++r) v[b + r * B] = lds[lds_slot<C>(base + r * NSPRE)];
    }
}

// The transposed engine: the stages of fft in reverse order, each transposed (DFTs, then
// twiddles) and the exchanges reversed.  The DFT matrix being symmetric, this is the same
// transform (INV: the inverse); it takes fft's output layout to fft's input layout: on entry
// thread t2 holds elements t2 + G e (area lds2), on exit thread t1 holds t1 + G e (area
// lds1), the roles switching at the last exchange.  With h = 1 it is the transpose of fft's
// twisted transform, i.e. the transform followed by the cropping twist y_j W_2N^{-j} (INV),
// whose constant part is applied last: the odd half of a cropped inverse without a separate
// twist.  The areas must not be in use by other threads when it is entered; WAVE as in fft.
template <class C, bool INV, bool WAVE = false>
__device__ __forceinline__ void fft_t(cpx (&v)[C::E], int t1, cpx* lds1, int t2, cpx* lds2,
                                      gp<const cpx> __restrict__ tw, int h) {
    constexpr int N = C::N;
    constexpr int E = C::E;
    constexpr int R0 = C::R[0], R1 = C::R[1], R2 = C::R[2], R3 = C::R[3];
    if constexpr (C::NS >= 4) {
        stage_compute_t<N, E, R3, R0 * R1 * R2, INV>(v, t2, tw, h);
        stage_ungather<C>(v, t2, lds2);
        lds_sync<WAVE>();
        stage_unscatter<C, R2, R0 * R1>(v, t2, lds2);
        lds_sync<WAVE>();
    }
    if constexpr (C::NS >= 3) {
        stage_compute_t<N, E, R2, R0 * R1, INV>(v, t2, tw, h);
        stage_ungather<C>(v, t2, lds2);
        lds_sync<WAVE>();
        stage_unscatter<C, R1, R0>(v, t2, lds2);
        lds_sync<WAVE>();
    }
    if constexpr (C::NS >= 2) {
        stage_compute_t<N, E, R1, R0, INV>(v, t2, tw, h);
        stage_ungather<C>(v, t2, lds2);
        lds_sync<WAVE>();
        stage_unscatter<C, R0, 1>(v, t1, lds1);
    }
    stage_compute_t<N, E, R0, 1, INV>(v, t1, tw, h);
    if (h) twist_const<C, INV>(v);
}

}  // namespace gsk
