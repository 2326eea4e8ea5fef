// host_plan.hpp -- plan-time host computations (Algorithm 1, "Precomputation").
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace gsh {

enum Kernel {
    COULOMB_3D = 0, COULOMB_2D = 1, POISSON_2D = 2, DIPOLAR_3D = 3, GAUSSIAN_SUM = 4, DAVEY_STEWARTSON_2D = 5,
    INVERSE_POWER = 6
};

// Gaussian sum U_GS(r) = sum_q w[q] exp(-tau[q]^2 r^2) in physical units; q = 0 is tau = 0.
struct Table {
    std::vector<double> w, tau;
    int S = 0;
    double delta = 0.0;   // physical near-field radius
    double beta = 0.0;    // exponent of the inverse-power kernel r^-beta
};

// Sinc-quadrature tables (Section 3) fitted on [delta_rel, hi] in units of the
// length Lu (the largest half-width of the box; hi = 2 |L| / Lu, the largest
// distance in the box: 2 sqrt(d) for a cube).  False when eps is not reachable.
bool coulomb_table(int d, double Lu, double hi, double delta_rel, double eps, Table& out);
bool poisson_table(double Lu, double hi, double delta_rel, double eps, Table& out);
// r^-beta (0 < beta < d): 2/Gamma(beta/2) int tau^(beta-1) exp(-r^2 tau^2) dtau with
// tau = exp(t - e^-t), step 2 ln(S)/S, negligible nodes dropped.
bool power_table(double beta, double Lu, double hi, double delta_rel, double eps, Table& out);

// Max error of the rescaled tables on their fit interval (for tests and reports).
double coulomb_table_error(int S, double lo, double hi);

// F[k*Q + q] = int_{-2L}^{2L} exp(-tau_q^2 y^2) cos(xi_k y) dy, k = 0..n, at the frequencies
// xi_k = pi k / (pad L) of the density padded to [-pad L, pad L] (pad = 2, or 3 for B_3).
void factors_1d(const std::vector<double>& tau, double L, int n, std::vector<double>& F, int pad = 2);

// Taylor constants of the near-field correction (Section 2.3).
void taylor_constants(int kernel, int d, const Table& t, double& A0, double& c2);

// Host assembly of the stored octant prod_i (n_i + 1), 1/prod_i (2 n_i) folded in.  Octant
// axes (kx, ky[, kz]): nk[i], Lk[i] and Fk[i] are the points, half-width and factors of axis
// x, y[, z].  dxx: multiply by -xi_x^2, the symbol of d_xx (Davey-Stewartson).  lapu: 0 for
// the Taylor term's Laplacian on the padded grid (weight 1), else the padding factor p and
// that Laplacian on the density's own grid (weight p^d at indices all divisible by p, where
// the padded transform is the density's n-point transform; 0 at the others).
void assemble_spectrum(int d, const int* nk, const double* Lk, const Table& t, const std::vector<double>* Fk,
                       double A0, double c2, bool dxx, int lapu, std::vector<double>& S);

// exp(-i pi m / n), m = 0..2n-1, as interleaved (re, im).
void twiddles(int n, std::vector<double>& tw);

}  // namespace gsh
