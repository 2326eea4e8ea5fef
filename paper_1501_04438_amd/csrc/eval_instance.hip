// eval_instance.hip -- launchers of the evaluation passes for one transform length.
// Compiled once per supported n with -DGS_N=<n>; the build lists the sizes.
#include "device_api.hpp"
#include "passes.hpp"
#include "sizes.hpp"

#ifndef GS_N
#error "GS_N must be defined"
#endif

#define GS_CAT2(a, b) a##b
#define GS_CAT(a, b) GS_CAT2(a, b)

namespace gsk {

// Persistent grid of the fused pass: `mult` rounds of co-resident blocks, at most one
// block per pencil group (plan default four rounds, the autotuner's choice at n = 256).
static inline unsigned fused_grid(int groups, int cap, int mult) {
    const long long c = (long long)(mult > 0 ? mult : 2) * cap;
    return (unsigned)((cap > 0 && groups > c) ? c : groups);
}

// Co-resident blocks of a kernel on the whole device (CUs x blocks per CU), computed once.
static int resident_blocks(const void* fn, int threads) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, 0) != hipSuccess) return 0;
    return cus * (per > 0 ? per : 1);
}

// Tile-shape variants of the cubic passes (bits of EvalArgs::tile_bits; none changes a bit
// of the result): x-forward pass bits 0-1 (0: the default row pairs per block, 1: twice as
// many), y passes bits 2-3 (0: default z-pencils per block, 1: half, 2: twice), fused pass
// bits 4-5 (0: default pencils per block, 1: half, 2: twice), x-inverse pass bits 6-7 (as
// the x-forward pass).  Compiled for the lengths gs_tile_variants
// names, where LDS allows; elsewhere every value selects the default.
constexpr int LDS_LIMIT = 160 * 1024;
template <int N> constexpr int px_of(int v) {
    constexpr int P = Geo<N>::PPX;
    // (whole tiles only: a tile that does not divide the grid would pair rows differently)
    return (gs_tile_variants(N) && v == 1 && 2 * P * Geo<N>::A * 16 <= LDS_LIMIT && N % (4 * P) == 0) ? 2 * P : P;
}
template <int N> constexpr int py_of(int v) {
    constexpr int P = Geo<N>::PPY;
    if (!gs_tile_variants(N)) return P;
    if (v == 1 && P >= 2) return P / 2;
    if (v == 2 && 2 * P * Geo<N>::A * 16 <= LDS_LIMIT && 2 * P * Geo<N>::G <= 1024) return 2 * P;
    return P;
}
template <int N> constexpr int pz_of(int v) {
    constexpr int P = Geo<N>::PPZ;
    if (!gs_tile_variants(N)) return P;
    if (v == 1 && P >= 2) return P / 2;
    if (v == 2 && 4 * P * Geo<N>::AZ * 16 <= LDS_LIMIT && 4 * P * Geo<N>::GZ <= 1024) return 2 * P;
    return P;
}

// P5 with row pairs PX per block on radix plan XV; with the energy, the total of the fused
// pass's pencil sums.
template <int PX, int XV = 0>
static hipError_t launch_x_inverse_v(const EvalArgs& a, hipStream_t s) {
    constexpr int N = GS_N;
    constexpr int T = p5_threads<N, PX, XV>();
    const cpx* const X1 = reinterpret_cast<const cpx*>(a.X1);
    const cpx* const tw = reinterpret_cast<const cpx*>(a.tw);
    const bool hint = (a.hint_bits >> 4) & 1;
    const dim3 gx((N + 2 * PX - 1) / (2 * PX), a.d == 3 ? N : 1);
    if (a.energy && a.oscale != 1.0) {
        if (hint) k_x_c2r<N, NT_P5, PX, true, XV><<<gx, T, 0, s>>>(X1, a.u, tw, a.oscale);
        else k_x_c2r<N, 0, PX, true, XV><<<gx, T, 0, s>>>(X1, a.u, tw, a.oscale);
    } else {
        if (hint) k_x_c2r<N, NT_P5, PX, false, XV><<<gx, T, 0, s>>>(X1, a.u, tw);
        else k_x_c2r<N, 0, PX, false, XV><<<gx, T, 0, s>>>(X1, a.u, tw);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.energy) return e;
    // the energy's pencil sums were written by the fused pass
    return launch_energy_total(a.epart, a.epencils, a.escale, a.energy, s);
}

// Padding to B_3 on a cubic transform grid (lengths 3n/2): P1 and P5 with the density and the
// potential at their own extents (a.px, a.py, a.pz), at the default tile.
static hipError_t launch_x_emb(const EvalArgs& a, hipStream_t s, int pass) {
    constexpr int N = GS_N;
    if constexpr (N % 3 == 0) {
        using Gm = Geo<N>;
        Ext ext;
        ext.nx = a.px;
        ext.ny = a.py;
        ext.nz = a.d == 3 ? a.pz : 1;
        if (ext.nx > N || ext.ny > N || ext.nz > (a.d == 3 ? N : 1)) return hipErrorInvalidValue;
        const cpx* const tw = reinterpret_cast<const cpx*>(a.tw);
        dim3 gx((N + 2 * Gm::PPX - 1) / (2 * Gm::PPX), a.d == 3 ? N : 1);
        if (pass == 1) {
            cpx* const X1 = reinterpret_cast<cpx*>(a.X1);
            if (a.hint_bits & 1) k_x_r2c_emb<N, NT_P1><<<gx, Gm::TX, 0, s>>>(a.rho, X1, tw, ext);
            else k_x_r2c_emb<N, 0><<<gx, Gm::TX, 0, s>>>(a.rho, X1, tw, ext);
            return hipGetLastError();
        }
        const cpx* const X1 = reinterpret_cast<const cpx*>(a.X1);
        constexpr int T = p5_threads<N, Gm::PPX>();
        const bool hint = (a.hint_bits >> 4) & 1;
        // the x-inverse pass only for the rows and planes that hold potential values
        gx.x = (ext.ny + 2 * Gm::PPX - 1) / (2 * Gm::PPX);
        gx.y = ext.nz;
        const bool sc = a.energy && a.oscale != 1.0;
        if (sc) {
            if (hint) k_x_c2r_emb<N, NT_P5, true><<<gx, T, 0, s>>>(X1, a.u, tw, ext, a.oscale);
            else k_x_c2r_emb<N, 0, true><<<gx, T, 0, s>>>(X1, a.u, tw, ext, a.oscale);
        } else {
            if (hint) k_x_c2r_emb<N, NT_P5, false><<<gx, T, 0, s>>>(X1, a.u, tw, ext, 1.0);
            else k_x_c2r_emb<N, 0, false><<<gx, T, 0, s>>>(X1, a.u, tw, ext, 1.0);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess || !a.energy) return e;
        return launch_energy_total(a.epart, a.epencils, a.escale, a.energy, s);
    } else {
        (void)a;
        (void)s;
        (void)pass;
        return hipErrorInvalidValue;
    }
}

// Tile bit 10 selects the x-inverse pass's radix-plan variant (XPlan<N, 1>, at the default row
// pairs per block; bits 6-7 then do not apply) where one is compiled.
static hipError_t launch_x_inverse(const EvalArgs& a, hipStream_t s) {
    constexpr int N = GS_N;
    if (a.emb) return launch_x_emb(a, s, 5);
    if constexpr (x_radix_variant<N>()) {
        if ((a.tile_bits >> 10) & 1) return launch_x_inverse_v<Geo<N>::PPX, 1>(a, s);
    }
    if (((a.tile_bits >> 6) & 3) == 1 && px_of<N>(1) != px_of<N>(0)) return launch_x_inverse_v<px_of<N>(1)>(a, s);
    return launch_x_inverse_v<px_of<N>(0)>(a, s);
}

template <int PX, int XV = 0>
static hipError_t launch_x_forward_v(const EvalArgs& a, hipStream_t s) {
    constexpr int N = GS_N;
    constexpr int T = PX * GeoX<N, XV>::G;
    const cpx* const tw = reinterpret_cast<const cpx*>(a.tw);
    cpx* const X1 = reinterpret_cast<cpx*>(a.X1);
    const dim3 gx((N + 2 * PX - 1) / (2 * PX), a.d == 3 ? N : 1);
    if ((a.hint_bits >> 0) & 1) k_x_r2c<N, NT_P1, PX, XV><<<gx, T, 0, s>>>(a.rho, X1, tw);
    else k_x_r2c<N, 0, PX, XV><<<gx, T, 0, s>>>(a.rho, X1, tw);
    return hipGetLastError();
}

// Tile bit 9: the x-forward pass's radix-plan variant, as bit 10 for the x-inverse pass.
static hipError_t launch_x_forward(const EvalArgs& a, hipStream_t s) {
    constexpr int N = GS_N;
    if (a.emb) return launch_x_emb(a, s, 1);
    if constexpr (x_radix_variant<N>()) {
        if ((a.tile_bits >> 9) & 1) return launch_x_forward_v<Geo<N>::PPX, 1>(a, s);
    }
    if ((a.tile_bits & 3) == 1 && px_of<N>(1) != px_of<N>(0)) return launch_x_forward_v<px_of<N>(1)>(a, s);
    return launch_x_forward_v<px_of<N>(0)>(a, s);
}

// y passes (3D) with PY z-pencils per block: 2 forward, 4 inverse.
template <int PY, int YV = 0>
static hipError_t launch_y_v(const EvalArgs& a, hipStream_t s, int pass) {
    constexpr int N = GS_N;
    cpx* const X1 = reinterpret_cast<cpx*>(a.X1);
    cpx* const X2 = reinterpret_cast<cpx*>(a.X2);
    const cpx* const tw = reinterpret_cast<const cpx*>(a.tw);
    // padding to B_3 in place (a.emb): the y-inverse pass only for the planes z < pz, the only
    // ones the x-inverse pass reads
    const int zs = (pass == 4 && a.emb) ? a.pz : N;
    const dim3 gy((zs + PY - 1) / PY, a.kxn);
    constexpr int T = PY * GeoX<N, YV>::G;
    const bool hint = (a.hint_bits >> (pass - 1)) & 1;
    if (pass == 2) {
        if (hint) k_y_fwd<N, NT_P2, PY, YV><<<gy, T, 0, s>>>(X1, X2, tw, a.kx0);
        else k_y_fwd<N, 0, PY, YV><<<gy, T, 0, s>>>(X1, X2, tw, a.kx0);
    } else {
        if (hint) k_y_inv<N, NT_P4, PY, YV><<<gy, T, 0, s>>>(X2, X1, tw, a.kx0);
        else k_y_inv<N, 0, PY, YV><<<gy, T, 0, s>>>(X2, X1, tw, a.kx0);
    }
    return hipGetLastError();
}

// Tile bits 11 (y-forward) and 12 (y-inverse) select the pass's radix-plan variant (XPlan<N, 1>
// at the default z-pencils per block; bits 2-3 then do not apply to that pass).
template <int N>
static hipError_t launch_y(const EvalArgs& a, hipStream_t s, int pass) {
    static_assert(N <= GS_MAX_N_3D, "the y passes run in 3D only");
    if constexpr (x_radix_variant<N>()) {
        if ((a.tile_bits >> (pass == 2 ? 11 : 12)) & 1) return launch_y_v<Geo<N>::PPY, 1>(a, s, pass);
    }
    const int v = (a.tile_bits >> 2) & 3;
    if (v == 1 && py_of<N>(1) != py_of<N>(0)) return launch_y_v<py_of<N>(1)>(a, s, pass);
    if (v == 2 && py_of<N>(2) != py_of<N>(0)) return launch_y_v<py_of<N>(2)>(a, s, pass);
    return launch_y_v<py_of<N>(0)>(a, s, pass);
}

// Fused pass with PZ pencils per block on radix plan RV (3D: persistent rounds at n = 256;
// 2D: one block per pencil group).  The energy instances exist for each plan's default tile.
template <int PZ, int RV = 0>
static hipError_t launch_fused_v(const EvalArgs& a, hipStream_t s, const DipoleArgs& dip) {
    constexpr int N = GS_N;
    constexpr int T = PZ * 2 * GeoZ<N, RV>::GZ;
    constexpr bool ETILE = (PZ == GeoZ<N, RV>::PPZ);
    const cpx* const tw = reinterpret_cast<const cpx*>(a.tw);
    const bool hint = (a.hint_bits >> 2) & 1;
    if constexpr (N <= GS_MAX_N_3D) {
      if (a.d == 3) {
        cpx* const X2 = reinterpret_cast<cpx*>(a.X2);
        static const int cap3 = resident_blocks((const void*)k_fused<N, 3, SPEC_PLAIN, 0, PZ, false, RV>, T);
        const int capf = a.max_blocks_fused > 0 ? a.max_blocks_fused : cap3;
        const int np = a.kxn * 2 * N;
        const int groups = (np + PZ - 1) / PZ;
        const unsigned nb = gs_fused_persistent(3, N) ? fused_grid(groups, capf, a.fused_grid_mult) : (unsigned)groups;
        if constexpr (ETILE) {
            if (a.energy) {
                // with the energy sum of every pencil (the default tile only)
                if (a.dipolar) {
                    if (hint) k_fused<N, 3, SPEC_DIPOLAR, NT_P3, PZ, true, RV><<<nb, T, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip, a.epart);
                    else k_fused<N, 3, SPEC_DIPOLAR, 0, PZ, true, RV><<<nb, T, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip, a.epart);
                } else {
                    if (hint) k_fused<N, 3, SPEC_PLAIN, NT_P3, PZ, true, RV><<<nb, T, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip, a.epart);
                    else k_fused<N, 3, SPEC_PLAIN, 0, PZ, true, RV><<<nb, T, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip, a.epart);
                }
                return hipGetLastError();
            }
        }
        if (a.dipolar) {
            if (hint) k_fused<N, 3, SPEC_DIPOLAR, NT_P3, PZ, false, RV><<<nb, T, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip);
            else k_fused<N, 3, SPEC_DIPOLAR, 0, PZ, false, RV><<<nb, T, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip);
        } else {
            if (hint) k_fused<N, 3, SPEC_PLAIN, NT_P3, PZ, false, RV><<<nb, T, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip);
            else k_fused<N, 3, SPEC_PLAIN, 0, PZ, false, RV><<<nb, T, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip);
        }
        return hipGetLastError();
      }
    }
    static_assert(!gs_fused_persistent(2, N), "the 2D fused pass runs one block per pencil group");
    cpx* const X1 = reinterpret_cast<cpx*>(a.X1);
    const int np = N + 1;
    const unsigned nb = (unsigned)((fused_slots<N, 2, RV>(np) + PZ - 1) / PZ);
    if constexpr (ETILE) {
        if (a.energy) {
            if (hint) k_fused<N, 2, SPEC_PLAIN, NT_P3, PZ, true, RV><<<nb, T, 0, s>>>(X1, a.spec, tw, np, 0, dip, a.epart);
            else k_fused<N, 2, SPEC_PLAIN, 0, PZ, true, RV><<<nb, T, 0, s>>>(X1, a.spec, tw, np, 0, dip, a.epart);
            return hipGetLastError();
        }
    }
    if (hint) k_fused<N, 2, SPEC_PLAIN, NT_P3, PZ, false, RV><<<nb, T, 0, s>>>(X1, a.spec, tw, np, 0, dip);
    else k_fused<N, 2, SPEC_PLAIN, 0, PZ, false, RV><<<nb, T, 0, s>>>(X1, a.spec, tw, np, 0, dip);
    return hipGetLastError();
}

// Tile bit 8 selects the fused pass's radix-plan variant (FusedPlan<N, 1>, at its own
// default pencils per block; bits 4-5 then do not apply) where one is compiled.
static hipError_t launch_fused(const EvalArgs& a, hipStream_t s, const DipoleArgs& dip) {
    constexpr int N = GS_N;
    if constexpr (fused_radix_variant<N>()) {
        if ((a.tile_bits >> 8) & 1) return launch_fused_v<GeoZ<N, 1>::PPZ, 1>(a, s, dip);
    }
    const int v = a.energy ? 0 : (a.tile_bits >> 4) & 3;
    if (v == 1 && pz_of<N>(1) != pz_of<N>(0)) return launch_fused_v<pz_of<N>(1)>(a, s, dip);
    if (v == 2 && pz_of<N>(2) != pz_of<N>(0)) return launch_fused_v<pz_of<N>(2)>(a, s, dip);
    return launch_fused_v<pz_of<N>(0)>(a, s, dip);
}

int GS_CAT(tile_variants_, GS_N)() {
    // bit 0: an x variant exists (either x pass); bits 1, 2: y half / double; bits 3, 4: fused
    // half / double; bit 5: a radix-plan variant of the fused pass; bit 6: of the x passes;
    // bit 7: of the y passes
    constexpr int N = GS_N;
    return (px_of<N>(1) != px_of<N>(0) ? 1 : 0) | (py_of<N>(1) != py_of<N>(0) ? 2 : 0) |
           (py_of<N>(2) != py_of<N>(0) ? 4 : 0) | (pz_of<N>(1) != pz_of<N>(0) ? 8 : 0) |
           (pz_of<N>(2) != pz_of<N>(0) ? 16 : 0) | (fused_radix_variant<N>() ? 32 : 0) |
           (x_radix_variant<N>() ? 64 : 0) | (x_radix_variant<N>() && N <= GS_MAX_N_3D ? 128 : 0);
}

// Pass `pass` of a grid whose axes have their own n, N being the length the pass transforms
// (x for passes 1 and 5, y for 2 and 4, the fused axis for 3: z in 3D, y in 2D).  One block
// per tile or pencil group; the cache-hint variants as in the cubic launches.
hipError_t GS_CAT(launch_eval_g_, GS_N)(const EvalArgs& a, hipStream_t s, int pass) {
    constexpr int N = GS_N;
    using Gm = Geo<N>;
    Ext ext;
    ext.nx = a.nx;
    ext.ny = a.ny;
    ext.nz = a.d == 3 ? a.nz : 1;
    cpx* const X1 = reinterpret_cast<cpx*>(a.X1);
    cpx* const X2 = reinterpret_cast<cpx*>(a.X2);
    const bool hint = (a.hint_bits >> (pass - 1)) & 1;
    if (pass == 1 || pass == 5) {
        const cpx* const tw = reinterpret_cast<const cpx*>(a.twx);
        const dim3 gx((ext.ny + 2 * Gm::PPX - 1) / (2 * Gm::PPX), ext.nz);
        if (pass == 1) {
            if (hint) k_x_r2c_g<N, NT_P1><<<gx, Gm::TX, 0, s>>>(a.rho, X1, tw, ext);
            else k_x_r2c_g<N, 0><<<gx, Gm::TX, 0, s>>>(a.rho, X1, tw, ext);
            return hipGetLastError();
        }
        if (a.energy && a.oscale != 1.0) {
            if (hint) k_x_c2r_g<N, NT_P5, true><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw, ext, a.oscale);
            else k_x_c2r_g<N, 0, true><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw, ext, a.oscale);
        } else {
            if (hint) k_x_c2r_g<N, NT_P5, false><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw, ext, 1.0);
            else k_x_c2r_g<N, 0, false><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw, ext, 1.0);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess || !a.energy) return e;
        // the energy's pencil sums were written by the fused pass
        return launch_energy_total(a.epart, a.epencils, a.escale, a.energy, s);
    }
    DipoleArgs dip;
    for (int i = 0; i < 3; ++i) {
        dip.dxi[i] = a.dxi[i];
        dip.cdiag[i] = a.cdiag[i];
        dip.ccross[i] = a.ccross[i];
    }
    dip.nm_over_M = a.nm_over_M;
    if constexpr (N <= GS_MAX_N_3D) {
      if (a.d == 3) {
        const cpx* const twy = reinterpret_cast<const cpx*>(a.twy);
        const dim3 gy((ext.nz + Gm::PPY - 1) / Gm::PPY, a.kxn);
        if (pass == 2) {
            if (hint) k_y_fwd_g<N, NT_P2><<<gy, Gm::TY, 0, s>>>(X1, X2, twy, a.kx0, ext);
            else k_y_fwd_g<N, 0><<<gy, Gm::TY, 0, s>>>(X1, X2, twy, a.kx0, ext);
        } else if (pass == 4) {
            if (hint) k_y_inv_g<N, NT_P4><<<gy, Gm::TY, 0, s>>>(X2, X1, twy, a.kx0, ext);
            else k_y_inv_g<N, 0><<<gy, Gm::TY, 0, s>>>(X2, X1, twy, a.kx0, ext);
        } else if (pass == 3) {
            const cpx* const twz = reinterpret_cast<const cpx*>(a.twz);
            const int np = a.kxn * 2 * ext.ny;
            const unsigned nb = (unsigned)((np + Gm::PPZ - 1) / Gm::PPZ);
            double* const ep = a.epart;
            if (a.dipolar) {
                if (a.energy) {
                    if (hint) k_fused_g<N, 3, SPEC_DIPOLAR, NT_P3, true><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext, ep);
                    else k_fused_g<N, 3, SPEC_DIPOLAR, 0, true><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext, ep);
                } else {
                    if (hint) k_fused_g<N, 3, SPEC_DIPOLAR, NT_P3><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext);
                    else k_fused_g<N, 3, SPEC_DIPOLAR, 0><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext);
                }
            } else {
                if (a.energy) {
                    if (hint) k_fused_g<N, 3, SPEC_PLAIN, NT_P3, true><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext, ep);
                    else k_fused_g<N, 3, SPEC_PLAIN, 0, true><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext, ep);
                } else {
                    if (hint) k_fused_g<N, 3, SPEC_PLAIN, NT_P3><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext);
                    else k_fused_g<N, 3, SPEC_PLAIN, 0><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext);
                }
            }
        } else {
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
      }
    }
    if (pass != 3 || a.d != 2) return hipErrorInvalidValue;
    const cpx* const twy = reinterpret_cast<const cpx*>(a.twy);
    const int np = ext.nx + 1;
    const unsigned nb = (unsigned)((fused_slots<N, 2>(np) + Gm::PPZ - 1) / Gm::PPZ);
    if (a.energy) {
        if (hint) k_fused_g<N, 2, SPEC_PLAIN, NT_P3, true><<<nb, Gm::TZ, 0, s>>>(X1, a.spec, twy, np, 0, dip, ext, a.epart);
        else k_fused_g<N, 2, SPEC_PLAIN, 0, true><<<nb, Gm::TZ, 0, s>>>(X1, a.spec, twy, np, 0, dip, ext, a.epart);
        return hipGetLastError();
    }
    if (hint) k_fused_g<N, 2, SPEC_PLAIN, NT_P3><<<nb, Gm::TZ, 0, s>>>(X1, a.spec, twy, np, 0, dip, ext);
    else k_fused_g<N, 2, SPEC_PLAIN, 0><<<nb, Gm::TZ, 0, s>>>(X1, a.spec, twy, np, 0, dip, ext);
    return hipGetLastError();
}

hipError_t GS_CAT(launch_eval_, GS_N)(const EvalArgs& a, hipStream_t s, int which) {
    constexpr int N = GS_N;
    DipoleArgs dip;
    for (int i = 0; i < 3; ++i) dip.dxi[i] = a.dxi[i];
    for (int i = 0; i < 3; ++i) {
        dip.cdiag[i] = a.cdiag[i];
        dip.ccross[i] = a.ccross[i];
    }
    dip.nm_over_M = a.nm_over_M;
    auto run = [&](int p) { return which < 0 || which == p; };
    hipError_t e = hipSuccess;
    if (run(1) && (e = launch_x_forward(a, s)) != hipSuccess) return e;
    if (a.d == 3) {
        if constexpr (N <= GS_MAX_N_3D) {
            if (run(2) && (e = launch_y<N>(a, s, 2)) != hipSuccess) return e;
            if (run(3) && (e = launch_fused(a, s, dip)) != hipSuccess) return e;
            if (run(4) && (e = launch_y<N>(a, s, 4)) != hipSuccess) return e;
        } else {
            return hipErrorInvalidValue;
        }
    } else if (run(3) && (e = launch_fused(a, s, dip)) != hipSuccess) {
        return e;
    }
    if (run(5)) return launch_x_inverse(a, s);
    return hipSuccess;
}

}  // namespace gsk
