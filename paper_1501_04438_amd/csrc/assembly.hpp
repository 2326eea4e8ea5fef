// assembly.hpp -- stored-spectrum assembly on the FP64 matrix cores (gfx950).
//
// The coefficient sums of Section 2.2 (eq. (tensor) summed with the weights as
// in eq. (I1FFT); eq. (tensor_ani) for rectangular boxes), with the Taylor terms
// of Section 2.3 folded in, on the octant k_j = 0..n of the padded frequencies
// xi_k = pi k / (2 L_j) of each axis:
//     S[k1][k2][k3] = ( sum_q (w_q Fx[k1][q]) Fy[k2][q] Fz[k3][q]
//                       + A0 - c2 (xi_k1^2 + xi_k2^2 + xi_k3^2) ) / prod_j (2 n_j)
// is a rank-Q contraction whose right operand is the Khatri-Rao product
// B[q][(k2,k3)] = Fy[k2][q] Fz[k3][q]: a GEMM of shape (nx+1) x Q x (ny+1)(nz+1) with
// B formed in registers.  2D: S[k1][k3] with B[q][k3] = Fy[k3][q] (passed as FC).
// dxx != 0 multiplies the result by -xi_k1^2, the symbol of d_xx (Davey-Stewartson
// potential: the Poisson spectrum applied to the second x-derivative of rho).
// lapu != 0 takes the Taylor term's Laplacian on the density's own grid (period 2L): on
// the padded grid of p n points (lapu = p, the padding factor) its symbol is p^d (-|xi|^2)
// at the indices whose every component is divisible by p (those are the n-point grid's
// frequencies, with the same xi) and 0 elsewhere, since the padded transform there is the
// n-point transform of rho.
//
// v_mfma_f64_16x16x4f64 operand layout (one wave, lane l = 0..63):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[(l / 16) + 4 r][l % 16] in element r = 0..3
// (the D layout was read off the hardware with a one-wave probe)
#pragma once

#include <hip/hip_runtime.h>

namespace gsk {

typedef double v4d __attribute__((ext_vector_type(4)));

// One wave computes a (16*MB) x 16 tile: MB row blocks of k1 against 16 columns.  n1, n1b,
// n1c: the octant extents of k1, k2, k3 (each axis its own n on rectangular grids).
template <int MB, int DIM>
__global__ void __launch_bounds__(256) k_assemble(const double* __restrict__ AT,   // [Qp][ldk]: w_q Fx[k][q]
                                                  const double* __restrict__ FB,   // [Qp][ldk]: factor of k2
                                                  const double* __restrict__ FC,   // [Qp][ldk]: factor of k3
                                                  int ldk, int n1, int n1b, int n1c, int Qp,
                                                  double* __restrict__ out,
                                                  double A0, double c2, double dx1, double dx2, double dx3,
                                                  double invM, int dxx, int lapu) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long ncols = (DIM == 3) ? (long)n1b * n1c : (long)n1c;
    const long col0 = ((long)blockIdx.x * 4 + wave) * 16;
    if (col0 >= ncols) return;                              // whole wave idle: uniform exit
    const int k1base = blockIdx.y * MB * 16;
    const int i = lane & 15, kk = lane >> 4;

    const long colb = (col0 + i < ncols) ? col0 + i : ncols - 1;
    const int k2 = (DIM == 3) ? (int)(colb / n1c) : 0;
    const int k3 = (DIM == 3) ? (int)(colb % n1c) : (int)colb;

    v4d acc[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = v4d{0.0, 0.0, 0.0, 0.0};

    // operands of K step q0 + 4 are loaded while the MFMAs of step q0 run (the last
    // step reloads its own rows)
    double a[MB], fb, fc;
    {
        const size_t row = (size_t)kk * ldk;
        fb = (DIM == 3) ? FB[row + k2] : 1.0;
        fc = FC[row + k3];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) a[mb] = AT[row + k1base + i + mb * 16];
    }
    for (int q0 = 0; q0 < Qp; q0 += 4) {
        const int qn = (q0 + 4 < Qp) ? q0 + 4 : q0;
        const size_t rown = (size_t)(qn + kk) * ldk;
        double an[MB];
        const double fbn = (DIM == 3) ? FB[rown + k2] : 1.0;
        const double fcn = FC[rown + k3];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) an[mb] = AT[rown + k1base + i + mb * 16];
        const double b = (DIM == 3) ? fb * fc : fc;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb], b, acc[mb], 0, 0, 0);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) a[mb] = an[mb];
        fb = fbn;
        fc = fcn;
    }

    const long c = col0 + (lane & 15);
    if (c < ncols) {
        double xs;
        bool even;            // k2 and k3 divisible by lapu (the unpadded-grid Laplacian lives there)
        const int lu = lapu ? lapu : 1;
        if constexpr (DIM == 3) {
            const double x2 = (double)(c / n1c) * dx2, x3 = (double)(c % n1c) * dx3;
            xs = x2 * x2 + x3 * x3;
            even = ((c / n1c) % lu == 0) && ((c % n1c) % lu == 0);
        } else {
            const double x3 = (double)c * dx3;
            xs = x3 * x3;
            even = (c % lu == 0);
        }
        const double lwe = (DIM == 3) ? (double)(lu * lu * lu) : (double)(lu * lu);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k1 = k1base + mb * 16 + kk + 4 * r;
                if (k1 < n1) {
                    const double x1 = (double)k1 * dx1;
                    const double f = dxx ? -(x1 * x1) * invM : invM;
                    // Laplacian weight: 1 on the padded grid; on the density's own grid
                    // p^d at indices all divisible by p, 0 elsewhere
                    const double lw = lapu ? ((even && (k1 % lu == 0)) ? lwe : 0.0) : 1.0;
                    out[(size_t)k1 * ncols + c] = (acc[mb][r] + A0 - c2 * lw * (x1 * x1 + xs)) * f;
                }
            }
        }
    }
}

}  // namespace gsk
