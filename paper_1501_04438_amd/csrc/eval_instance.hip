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

// P5, with the energy sum when the arguments ask for it.
static hipError_t launch_x_inverse(const EvalArgs& a, hipStream_t s, dim3 gx) {
    constexpr int N = GS_N;
    using Gm = Geo<N>;
    const cpx* const X1 = reinterpret_cast<const cpx*>(a.X1);
    const cpx* const tw = reinterpret_cast<const cpx*>(a.tw);
    const bool hint = (a.hint_bits >> 4) & 1;
    if (a.energy) {
        if (hint) k_x_c2r_energy<N, NT_P5><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw, a.rho, a.epart);
        else k_x_c2r_energy<N, 0><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw, a.rho, a.epart);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_energy_finish(a.epart, (int)(gx.x * gx.y), a.escale, a.energy, s);
    }
    if (hint) k_x_c2r<N, NT_P5><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw);
    else k_x_c2r<N, 0><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw);
    return hipGetLastError();
}

int GS_CAT(energy_blocks_, GS_N)(int d) {
    constexpr int N = GS_N;
    return (N + 2 * Geo<N>::PPX - 1) / (2 * Geo<N>::PPX) * (d == 3 ? N : 1);
}

// Rectangular grids (each axis its own n): x-pass blocks when N is the x length.
int GS_CAT(energy_blocks_g_, GS_N)(int ny, int nz) {
    constexpr int N = GS_N;
    return (ny + 2 * Geo<N>::PPX - 1) / (2 * Geo<N>::PPX) * nz;
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
        if (a.energy) {
            if (hint) k_x_c2r_g<N, NT_P5, true><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw, a.rho, a.epart, ext);
            else k_x_c2r_g<N, 0, true><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw, a.rho, a.epart, ext);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            return launch_energy_finish(a.epart, (int)(gx.x * gx.y), a.escale, a.energy, s);
        }
        if (hint) k_x_c2r_g<N, NT_P5, false><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw, nullptr, nullptr, ext);
        else k_x_c2r_g<N, 0, false><<<gx, Gm::TX, 0, s>>>(X1, a.u, tw, nullptr, nullptr, ext);
        return hipGetLastError();
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
            if (a.dipolar) {
                if (hint) k_fused_g<N, 3, SPEC_DIPOLAR, NT_P3><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext);
                else k_fused_g<N, 3, SPEC_DIPOLAR, 0><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext);
            } else {
                if (hint) k_fused_g<N, 3, SPEC_PLAIN, NT_P3><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext);
                else k_fused_g<N, 3, SPEC_PLAIN, 0><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, twz, np, a.kx0, dip, ext);
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
    const unsigned nb = (unsigned)((np + Gm::PPZ - 1) / Gm::PPZ);
    if (hint) k_fused_g<N, 2, SPEC_PLAIN, NT_P3><<<nb, Gm::TZ, 0, s>>>(X1, a.spec, twy, np, 0, dip, ext);
    else k_fused_g<N, 2, SPEC_PLAIN, 0><<<nb, Gm::TZ, 0, s>>>(X1, a.spec, twy, np, 0, dip, ext);
    return hipGetLastError();
}

hipError_t GS_CAT(launch_eval_, GS_N)(const EvalArgs& a, hipStream_t s, int which) {
    constexpr int N = GS_N;
    using Gm = Geo<N>;
    DipoleArgs dip;
    for (int i = 0; i < 3; ++i) dip.dxi[i] = a.dxi[i];
    for (int i = 0; i < 3; ++i) {
        dip.cdiag[i] = a.cdiag[i];
        dip.ccross[i] = a.ccross[i];
    }
    dip.nm_over_M = a.nm_over_M;
    const int nz = (a.d == 3) ? N : 1;
    cpx* const X1 = reinterpret_cast<cpx*>(a.X1);
    cpx* const X2 = reinterpret_cast<cpx*>(a.X2);
    const cpx* const tw = reinterpret_cast<const cpx*>(a.tw);
    static const int cap3 = resident_blocks((const void*)k_fused<N, 3, SPEC_PLAIN>, Gm::TZ);
    const int capf = a.max_blocks_fused > 0 ? a.max_blocks_fused : cap3;
    const dim3 gx((N + 2 * Gm::PPX - 1) / (2 * Gm::PPX), nz);
    auto run = [&](int p) { return which < 0 || which == p; };
    auto hint = [&](int p) { return (a.hint_bits >> (p - 1)) & 1; };
    const int fm = a.fused_grid_mult;
    if (run(1)) {
        if (hint(1)) k_x_r2c<N, NT_P1><<<gx, Gm::TX, 0, s>>>(a.rho, X1, tw);
        else k_x_r2c<N, 0><<<gx, Gm::TX, 0, s>>>(a.rho, X1, tw);
    }
    if constexpr (N <= GS_MAX_N_3D) {
      if (a.d == 3) {
        const dim3 gy((N + Gm::PPY - 1) / Gm::PPY, a.kxn);
        const int np = a.kxn * 2 * N;
        if (run(2)) {
            if (hint(2)) k_y_fwd<N, NT_P2><<<gy, Gm::TY, 0, s>>>(X1, X2, tw, a.kx0);
            else k_y_fwd<N, 0><<<gy, Gm::TY, 0, s>>>(X1, X2, tw, a.kx0);
        }
        if (run(3)) {
            const int groups = (np + Gm::PPZ - 1) / Gm::PPZ;
            const unsigned nb = gs_fused_persistent(3, N) ? fused_grid(groups, capf, fm) : (unsigned)groups;
            if (a.dipolar) {
                if (hint(3)) k_fused<N, 3, SPEC_DIPOLAR, NT_P3><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip);
                else k_fused<N, 3, SPEC_DIPOLAR, 0><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip);
            } else {
                if (hint(3)) k_fused<N, 3, SPEC_PLAIN, NT_P3><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip);
                else k_fused<N, 3, SPEC_PLAIN, 0><<<nb, Gm::TZ, 0, s>>>(X2, a.spec, tw, np, a.kx0, dip);
            }
        }
        if (run(4)) {
            if (hint(4)) k_y_inv<N, NT_P4><<<gy, Gm::TY, 0, s>>>(X2, X1, tw, a.kx0);
            else k_y_inv<N, 0><<<gy, Gm::TY, 0, s>>>(X2, X1, tw, a.kx0);
        }
        if (run(5)) return launch_x_inverse(a, s, gx);
        return hipGetLastError();
      }
    }
    if (run(3)) {
        static_assert(!gs_fused_persistent(2, N), "the 2D fused pass runs one block per pencil group");
        const int np = N + 1;
        const unsigned nb = (unsigned)((np + Gm::PPZ - 1) / Gm::PPZ);
        if (hint(3)) k_fused<N, 2, SPEC_PLAIN, NT_P3><<<nb, Gm::TZ, 0, s>>>(X1, a.spec, tw, np, 0, dip);
        else k_fused<N, 2, SPEC_PLAIN, 0><<<nb, Gm::TZ, 0, s>>>(X1, a.spec, tw, np, 0, dip);
    }
    if (run(5)) return launch_x_inverse(a, s, gx);
    return hipGetLastError();
}

}  // namespace gsk
