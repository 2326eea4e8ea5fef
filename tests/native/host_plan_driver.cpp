// Host-side plan computations run under the address and undefined-behaviour sanitizers
// (built and run by tests/test_host_sanitizers.py with g++): Gaussian-sum tables, factor
// integrals, Taylor constants, the host spectrum assembly and the twiddle table, on small
// cubic and rectangular grids.  Prints one line per case for the test to compare.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_1501_04438_amd/csrc/host_plan.hpp"

using namespace gsh;

static double checksum(const std::vector<double>& v) {
    double s = 0.0;
    for (size_t i = 0; i < v.size(); ++i) s += v[i] * (1.0 + 1e-3 * (double)(i % 97));
    return s;
}

static int run(const char* name, int kernel, int d, int n, const double* Lk, double eps, double beta) {
    double Lu = 0.0, sum2 = 0.0;
    for (int i = 0; i < d; ++i) Lu = std::fmax(Lu, Lk[i]);
    for (int i = 0; i < d; ++i) sum2 += (Lk[i] / Lu) * (Lk[i] / Lu);
    const double hi = 2.0 * std::sqrt(sum2);
    Table t;
    bool ok;
    if (kernel == POISSON_2D || kernel == DAVEY_STEWARTSON_2D) ok = poisson_table(Lu, hi, 1e-4, eps, t);
    else if (kernel == INVERSE_POWER) ok = power_table(beta, Lu, hi, 1e-4, eps, t);
    else ok = coulomb_table(d, Lu, hi, 1e-4, eps, t);
    if (!ok) {
        std::printf("%s table-failed\n", name);
        return 1;
    }
    std::vector<double> Fk[3];
    for (int i = 0; i < d; ++i) factors_1d(t.tau, Lk[i], n, Fk[i]);
    double A0 = 0.0, c2 = 0.0;
    taylor_constants(kernel, d, t, A0, c2);
    std::vector<double> S;
    const int nk[3] = {n, n, n};
    assemble_spectrum(d, nk, Lk, t, Fk, A0, c2, kernel == DAVEY_STEWARTSON_2D, false, S);
    std::vector<double> tw;
    twiddles(n, tw);
    std::printf("%s S=%d Q=%zu A0=%.17g c2=%.17g spec0=%.17g specsum=%.17g tw=%zu\n", name, t.S, t.w.size(), A0, c2,
                S[0], checksum(S), tw.size());
    return 0;
}

int main() {
    const double cube3[3] = {4.0, 4.0, 4.0}, rect3[3] = {5.0, 4.0, 3.0}, rect2[2] = {9.0, 6.0};
    int bad = 0;
    bad += run("coulomb3d", COULOMB_3D, 3, 12, cube3, 1e-14, 0.0);
    bad += run("coulomb3d_rect", COULOMB_3D, 3, 12, rect3, 1e-14, 0.0);
    bad += run("poisson2d_rect", POISSON_2D, 2, 24, rect2, 1e-13, 0.0);
    bad += run("ds2d", DAVEY_STEWARTSON_2D, 2, 24, rect2, 1e-13, 0.0);
    bad += run("power3d", INVERSE_POWER, 3, 12, rect3, 1e-14, 0.7);
    return bad;
}
