// host_plan.cpp -- plan-time host computations (Algorithm 1, "Precomputation").
//
//  * Gaussian-sum tables by sinc quadrature (Section 3): 1/r from its Gaussian
//    integral with tau = sinh(t) (Section 3.2), ln r from Frullani's integral with
//    s = ln(1 + exp(sinh t)) (Section 3.3, read as described at poisson_table),
//    step theta = c0 ln(S)/S with c0 = 2.1 and 1 (Remark in Section 3.1), and S the
//    smallest value meeting eps on the fit interval; inverse powers r^-beta (the
//    Remark after eq. (GauInte)) with tau = exp(t - e^-t), c0 = 2 (power_table).
//  * One-dimensional factor integrals of the tensor-product coefficients
//    (Section 2.2, eq. (tensor)) on the box [-2L, 2L] at xi_k = pi k/(2L).
//  * Taylor constants A0, c2 of the near-field correction (Section 2.3).
//  * A host assembly of the stored spectrum (used for host-only plans and as
//    the reference of the device assembly), and the FFT twiddle table.
#include "host_plan.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>

namespace gsh {

static const double PI = 3.14159265358979323846;

static void parallel_for(int count, const std::function<void(int, int)>& body) {
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<unsigned>(hw ? hw : 1, 16);
    nt = std::max(1, std::min(nt, count));
    if (nt == 1) {
        body(0, count);
        return;
    }
    std::vector<std::thread> th;
    const int chunk = (count + nt - 1) / nt;
    for (int i = 0; i < nt; ++i) {
        const int lo = i * chunk, hi = std::min(count, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back(body, lo, hi);
    }
    for (auto& t : th) t.join();
}

// ------------------------------------------------------------------ sinc tables

static const int NPTS = 100001;   // check points on the fit interval (log spaced)

static std::vector<double> log_points(double lo, double hi) {
    std::vector<double> p(NPTS);
    const double a = std::log(lo), b = std::log(hi);
    for (int i = 0; i < NPTS; ++i) p[i] = std::exp(a + (b - a) * ((double)i / (NPTS - 1)));
    p[0] = lo;
    p[NPTS - 1] = hi;
    return p;
}

// max over the points with index multiple of `step` of f(point); threads for the full set
static double max_err(const std::vector<double>& pts, int step, const std::function<double(double)>& f) {
    const int cnt = (NPTS - 1) / step + 1;
    if (cnt < 4096) {
        double m = 0.0;
        for (int i = 0; i < cnt; ++i) m = std::max(m, f(pts[(size_t)i * step]));
        return m;
    }
    double best = 0.0;
    std::mutex mu;
    parallel_for(cnt, [&](int lo, int hi) {
        double m = 0.0;
        for (int i = lo; i < hi; ++i) m = std::max(m, f(pts[(size_t)i * step]));
        std::lock_guard<std::mutex> g(mu);
        best = std::max(best, m);
    });
    return best;
}

static void coulomb_nodes(int S, std::vector<double>& w, std::vector<double>& tau) {
    const double th = 2.1 * std::log((double)S) / S;
    w.assign(S + 1, 0.0);
    tau.assign(S + 1, 0.0);
    w[0] = th / std::sqrt(PI);
    for (int k = 1; k <= S; ++k) {
        w[k] = 2.0 * th * std::cosh(k * th) / std::sqrt(PI);
        tau[k] = std::sinh(k * th);
    }
}

static double coulomb_err_at(const std::vector<double>& w, const std::vector<double>& tau, double r) {
    double acc = 0.0;
    for (int q = (int)w.size() - 1; q >= 0; --q) acc += w[q] * std::exp(-(tau[q] * r) * (tau[q] * r));
    return std::fabs(1.0 - r * acc);
}

double coulomb_table_error(int S, double lo, double hi) {
    std::vector<double> w, tau;
    coulomb_nodes(S, w, tau);
    auto pts = log_points(lo, hi);
    return max_err(pts, 1, [&](double r) { return coulomb_err_at(w, tau, r); });
}

static const int S_MAX = 4000;

// Smallest S whose error on all NPTS points is <= eps: two cheap necessary
// tests on point subsets (every 1000th, every 50th) before the full check.
// Gives up (-1) once the coarse error has not improved for 200 consecutive S
// past S = 100: the rounding floor of the table lies above eps.
template <class ErrFn>
static int smallest_S(const std::vector<double>& pts, double eps, ErrFn err_for_S) {
    double best = 1e300;
    int best_at = 0;
    for (int S = 2; S <= S_MAX; ++S) {
        const double coarse = err_for_S(S, 1000);
        if (coarse < best) {
            best = coarse;
            best_at = S;
        } else if (S > 100 && S - best_at > 200) {
            break;
        }
        if (coarse > eps) continue;
        if (err_for_S(S, 50) > eps) continue;
        if (err_for_S(S, 1) <= eps) return S;
    }
    (void)pts;
    return -1;
}

struct TableKey {
    int kind;
    double hi, delta_rel, eps, beta;
    bool operator<(const TableKey& o) const {
        return std::tie(kind, hi, delta_rel, eps, beta) < std::tie(o.kind, o.hi, o.delta_rel, o.eps, o.beta);
    }
};
static std::mutex g_cache_mu;
static std::map<TableKey, int> g_S_cache;

bool coulomb_table(int d, double L, double hi, double delta_rel, double eps, Table& out) {
    const double lo = delta_rel;
    int S;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto it = g_S_cache.find({0, hi, delta_rel, eps, 0.0});
        S = (it == g_S_cache.end()) ? 0 : it->second;
    }
    if (S == 0) {
        auto pts = log_points(lo, hi);
        std::vector<double> w, tau;
        S = smallest_S(pts, eps, [&](int s, int step) {
            coulomb_nodes(s, w, tau);
            return max_err(pts, step, [&](double r) { return coulomb_err_at(w, tau, r); });
        });
        std::lock_guard<std::mutex> g(g_cache_mu);
        g_S_cache[{0, hi, delta_rel, eps, 0.0}] = S;
    }
    if (S < 0) return false;
    std::vector<double> w, tau;
    coulomb_nodes(S, w, tau);
    const double kappa = (d == 3) ? 1.0 / (4.0 * PI) : 1.0 / (2.0 * PI);
    out.S = S;
    out.delta = delta_rel * L;
    out.w.resize(w.size());
    out.tau.resize(w.size());
    for (size_t q = 0; q < w.size(); ++q) {
        out.w[q] = kappa * w[q] / L;
        out.tau[q] = tau[q] / L;
    }
    return true;
}

// r^-beta ~= sum_k w_k exp(-tau_k^2 r^2), nodes t_k = k theta, k = -S..S, theta = 2 ln(S)/S,
// tau_k = exp(t_k - e^-t_k), w_k = (2/Gamma(beta/2)) theta tau_k^beta (1 + e^-t_k); nodes whose
// largest relative contribution on [lo, hi] (at r = sqrt(beta/2)/tau clipped to it) is at most
// 1e-3 eps are dropped.  Sorted by increasing tau.
static void power_nodes(double beta, int S, double lo, double hi, double eps, std::vector<double>& w,
                        std::vector<double>& tau) {
    const double th = 2.0 * std::log((double)S) / S;
    const double g = 2.0 / std::tgamma(beta / 2.0);
    w.clear();
    tau.clear();
    for (int k = -S; k <= S; ++k) {
        const double t = k * th, em = std::exp(-t);
        const double tk = std::exp(t - em);
        const double wk = g * th * std::pow(tk, beta) * (1.0 + em);
        double rs = tk > 0.0 ? std::sqrt(beta / 2.0) / tk : hi;
        rs = std::min(hi, std::max(lo, rs));
        if (!(wk * std::pow(rs, beta) * std::exp(-(tk * rs) * (tk * rs)) > 1e-3 * eps)) continue;
        w.push_back(wk);
        tau.push_back(tk);
    }
}

static double power_err_at(double beta, const std::vector<double>& w, const std::vector<double>& tau, double r) {
    double acc = 0.0;
    for (int q = (int)w.size() - 1; q >= 0; --q) acc += w[q] * std::exp(-(tau[q] * r) * (tau[q] * r));
    return std::fabs(1.0 - std::pow(r, beta) * acc);
}

bool power_table(double beta, double L, double hi, double delta_rel, double eps, Table& out) {
    const double lo = delta_rel;
    int S;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto it = g_S_cache.find({2, hi, delta_rel, eps, beta});
        S = (it == g_S_cache.end()) ? 0 : it->second;
    }
    if (S == 0) {
        auto pts = log_points(lo, hi);
        std::vector<double> w, tau;
        S = smallest_S(pts, eps, [&](int s, int step) {
            power_nodes(beta, s, lo, hi, eps, w, tau);
            return max_err(pts, step, [&](double r) { return power_err_at(beta, w, tau, r); });
        });
        std::lock_guard<std::mutex> g(g_cache_mu);
        g_S_cache[{2, hi, delta_rel, eps, beta}] = S;
    }
    if (S < 0) return false;
    std::vector<double> w, tau;
    power_nodes(beta, S, lo, hi, eps, w, tau);
    out.S = S;
    out.beta = beta;
    out.delta = delta_rel * L;
    out.w.resize(w.size());
    out.tau.resize(w.size());
    const double scale = std::pow(L, -beta);
    for (size_t q = 0; q < w.size(); ++q) {
        out.w[q] = w[q] * scale;
        out.tau[q] = tau[q] / L;
    }
    return true;
}

// ln x ~= C0 - sum_k wh_k exp(-s_k x^2) on x in [1, X] (rescaled), nodes k = -S..S
// with negligible contributions (a_k X^2/2 <= 1e-3 eps) dropped.
static void poisson_nodes(int S, double X, double eps, double& C0, std::vector<double>& wh,
                          std::vector<double>& s) {
    const double th = 1.0 * std::log((double)S) / S;
    wh.clear();
    s.clear();
    for (int k = -S; k <= S; ++k) {
        const double t = k * th, sh = std::sinh(t);
        const double e = std::exp(-std::fabs(sh));
        const double sk = (sh > 0) ? sh + std::log1p(e) : std::log1p(e);
        const double sig = (sh >= 0) ? 1.0 / (1.0 + e) : e / (1.0 + e);
        const double a = th * std::cosh(t) * sig;
        if (!(a * X * X / 2.0 > 1e-3 * eps)) continue;
        wh.push_back(a / (2.0 * sk));
        s.push_back(sk);
    }
    C0 = 0.0;
    for (size_t q = 0; q < wh.size(); ++q) C0 += wh[q] * std::exp(-s[q]);
}

// |ln x - (C0 - sum_k wh_k exp(-s_k x^2))| summed as sum_k wh_k (exp(-s_k) - exp(-s_k x^2)):
// positive terms without cancellation against C0, so S follows the quadrature error.
static double poisson_err_at(double C0, const std::vector<double>& wh, const std::vector<double>& s, double x) {
    (void)C0;
    const double x2m1 = x * x - 1.0;
    double acc = 0.0;
    for (int q = (int)wh.size() - 1; q >= 0; --q) acc += wh[q] * (-std::exp(-s[q]) * std::expm1(-s[q] * x2m1));
    return std::fabs(std::log(x) - acc);
}

bool poisson_table(double L, double hi, double delta_rel, double eps, Table& out) {
    const double X = hi / delta_rel;
    int S;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto it = g_S_cache.find({1, hi, delta_rel, eps, 0.0});
        S = (it == g_S_cache.end()) ? 0 : it->second;
    }
    if (S == 0) {
        auto pts = log_points(1.0, X);
        double C0;
        std::vector<double> wh, s;
        S = smallest_S(pts, eps, [&](int ss, int step) {
            poisson_nodes(ss, X, eps, C0, wh, s);
            return max_err(pts, step, [&](double x) { return poisson_err_at(C0, wh, s, x); });
        });
        std::lock_guard<std::mutex> g(g_cache_mu);
        g_S_cache[{1, hi, delta_rel, eps, 0.0}] = S;
    }
    if (S < 0) return false;
    double C0;
    std::vector<double> wh, s;
    poisson_nodes(S, X, eps, C0, wh, s);
    const double delta = delta_rel * L;
    out.S = S;
    out.delta = delta;
    out.w.assign(1, -(std::log(delta) + C0) / (2.0 * PI));
    out.tau.assign(1, 0.0);
    for (size_t q = 0; q < wh.size(); ++q) {
        out.w.push_back(wh[q] / (2.0 * PI));
        out.tau.push_back(std::sqrt(s[q]) / delta);
    }
    return true;
}

// ------------------------------------------------------------------ factor integrals

static const int GL_M = 16;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration in long double.
static void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w) {
    x.resize(m);
    w.resize(m);
    for (int i = 0; i < m; ++i) {
        long double z = std::cos(PI * (i + 0.75) / (m + 0.5)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= m; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (z * p1 - p0) / (z * z - 1);
            long double dz = p1 / dp;
            z -= dz;
            if (std::fabs((double)dz) < 1e-19) break;
        }
        long double p0 = 1, p1 = z;
        for (int k = 2; k <= m; ++k) {
            long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = m * (z * p1 - p0) / (z * z - 1);
        x[i] = (double)z;
        w[i] = (double)(2.0L / ((1 - z * z) * dp * dp));
    }
}

// tau c >= 6.5: the truncation of the Gaussian at |y| = c is below 1e-19 relative
static const double TAU_C_CLOSED = 6.5;
// tau c <= 0.05: the power series of exp(-tau^2 y^2) in tau^2 with the exact cosine moments
static const double TAU_C_SERIES = 0.05;

// Neumaier's compensated summation: s + e carries the sum to about one rounding of s.
struct CompSum {
    double s = 0.0, e = 0.0;
    void add(double x) {
        const double t = s + x;
        e += (std::fabs(s) >= std::fabs(x)) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    double value() const { return s + e; }
};

// Small tau c: g(tau, xi_k) = sum_i (-tau^2)^i / i! M_2i(k) with the exact moments
// M_2i(k) = int_{-c}^{c} y^2i cos(xi_k y) dy = c^(2i+1) m_2i(a), a = xi_k c = 2 pi k / pad,
//   m_2i(0) = 2 / (2i + 1),
//   m_0(a) = 2 sin a / a, m_2i(a) = 2 sin a / a + (4i cos a - 2i (2i - 1) m_2i-2(a)) / a^2,
// by parts twice (sin a = 0 for pad = 2, a = pi k).  For tau c <= 0.05 the recurrence's
// growth at small k, (2i)!/a^2i, is outweighed by the series weight (tau c)^2i / i!: each
// term is exact to a few roundings of itself, and ten terms reach below 1e-25 relative.
static void factor_series(double t, double c, int n, int pad, int Q, int q, std::vector<double>& F) {
    const long double tc2 = (long double)t * t * c * c;
    for (int k = 0; k <= n; ++k) {
        // a = pi r / pad with r = 2k mod 2 pad: cos and sin exact where r / pad is whole
        const int r = (2 * k) % (2 * pad);
        const long double a = 2.0L * (long double)PI * k / pad, a2 = a * a;
        const long double ang = 3.141592653589793238462643383279502884L * r / pad;
        const long double cosa = (r % pad == 0) ? ((r == 0) ? 1.0L : -1.0L) : cosl(ang);
        const long double s2a = (r % pad == 0 || k == 0) ? 0.0L : 2.0L * sinl(ang) / a;   // 2 sin a / a
        long double m = (k == 0) ? 2.0L : s2a;           // m_0
        long double coef = 1.0L, sum = 0.0L;             // (-tau^2 c^2)^i / i!
        for (int i = 0; i < 10; ++i) {
            sum += coef * m;
            const int j = 2 * (i + 1);                  // next moment index
            m = (k == 0) ? 2.0L / (j + 1) : s2a + (2.0L * j * cosa - (long double)j * (j - 1) * m) / a2;
            coef *= -tc2 / (i + 1);
        }
        F[(size_t)k * Q + q] = (double)(sum * c);
    }
}

void factors_1d(const std::vector<double>& tau, double L, int n, std::vector<double>& F, int pad) {
    const int Q = (int)tau.size();
    const double c = 2.0 * L;
    F.assign((size_t)(n + 1) * Q, 0.0);
    std::vector<int> mid;
    for (int q = 0; q < Q; ++q) {
        const double t = tau[q];
        if (t == 0.0) {
            // 2 sin(xi_k c) / xi_k: 2c at k = 0; exactly 0 for pad = 2 (xi_k c = pi k)
            F[q] = 2.0 * c;
            for (int k = 1; k <= n; ++k) {
                const int r = (2 * k) % (2 * pad);
                if (r % pad == 0) continue;
                const double xi = 2.0 * PI * k / (pad * c);
                F[(size_t)k * Q + q] =
                    (double)(2.0L * sinl(3.141592653589793238462643383279502884L * r / pad)) / xi;
            }
        } else if (t * c >= TAU_C_CLOSED) {
            for (int k = 0; k <= n; ++k) {
                const double xi = 2.0 * PI * k / (pad * c);
                F[(size_t)k * Q + q] = std::sqrt(PI) / t * std::exp(-(xi * xi) / (4.0 * t * t));
            }
        } else if (t * c <= TAU_C_SERIES) {
            factor_series(t, c, n, pad, Q, q, F);
        } else {
            mid.push_back(q);
        }
    }
    if (mid.empty()) return;
    // Composite Gauss-Legendre on [0, c] (even integrand, factor 2): P = max(2n / pad, 8)
    // panels of GL_M nodes, at most one half-period of cos(xi_k y) per panel.  At node
    // y = c (p + s)/P the phase 2 pi k (p + s)/(pad P) is split into an exactly reduced
    // integer part pi ((2 k p) mod 2 pad P)/(pad P) and a part 2 pi k s/(pad P) <= pi.
    // The panel contributions are summed with compensation (up to 2048 panels).
    const int P = std::max(2 * n / pad, 8);
    const int Qm = (int)mid.size();
    std::vector<double> xg, wg;
    gauss_legendre(GL_M, xg, wg);
    std::vector<double> s(GL_M);
    for (int i = 0; i < GL_M; ++i) s[i] = 0.5 * (xg[i] + 1.0);
    const double hp = c / P;
    std::vector<double> gw((size_t)P * Qm * GL_M);    // [p][q][i]
    for (int p = 0; p < P; ++p)
        for (int qi = 0; qi < Qm; ++qi) {
            const double t = tau[mid[qi]];
            for (int i = 0; i < GL_M; ++i) {
                const double y = hp * (p + s[i]);
                gw[((size_t)p * Qm + qi) * GL_M + i] = hp * wg[i] * std::exp(-(t * y) * (t * y));
            }
        }
    const int R = 2 * pad * P;                       // phase period in units of pi / (pad P)
    std::vector<double> cosA(R), sinA(R);
    for (int m = 0; m < R; ++m) {
        const long double a = 3.141592653589793238462643383279502884L * (long double)m / (long double)(pad * P);
        cosA[m] = (double)cosl(a);
        sinA[m] = (double)sinl(a);
    }
    parallel_for(n + 1, [&](int k0, int k1) {
        std::vector<CompSum> acc(Qm);
        std::vector<double> cb(GL_M), sb(GL_M);
        for (int k = k0; k < k1; ++k) {
            for (int i = 0; i < GL_M; ++i) {
                const long double B =
                    3.141592653589793238462643383279502884L * ((long double)(2 * k) * s[i]) / (pad * P);
                cb[i] = (double)cosl(B);
                sb[i] = (double)sinl(B);
            }
            std::fill(acc.begin(), acc.end(), CompSum());
            for (int p = 0; p < P; ++p) {
                const int m = (int)(((long long)2 * k * p) % R);
                const double ca = cosA[m], sa = sinA[m];
                const double* g = &gw[(size_t)p * Qm * GL_M];
                for (int qi = 0; qi < Qm; ++qi) {
                    double dc = 0.0, ds = 0.0;
                    for (int i = 0; i < GL_M; ++i) {
                        dc += g[qi * GL_M + i] * cb[i];
                        ds += g[qi * GL_M + i] * sb[i];
                    }
                    acc[qi].add(ca * dc - sa * ds);
                }
            }
            for (int qi = 0; qi < Qm; ++qi) F[(size_t)k * Q + mid[qi]] = acc[qi].value();
        }
    });
}

// ------------------------------------------------------------------ Taylor constants

// A0 and c2 are small differences of moments (for the ln kernel c2 is about 1e-6 of the
// moments it is formed from: the Gaussian sum follows U deep into the ball), so the
// moments and their sums are formed in extended precision (x86 long double, 64-bit
// significand) and rounded once.
typedef long double ld;
static const ld PI_L = 3.141592653589793238462643383279502884L;

// gamma_m(tau) = int_0^delta r^m exp(-tau^2 r^2) dr, m = 1..4, without cancellation:
// a power series in u = tau delta for u <= 3 (largest term e^9, four of the nineteen
// digits), the closed forms through the incomplete gamma function otherwise
// (gamma_m = gammainc((m+1)/2, u^2) / (2 tau^(m+1)); the subtracted terms are below
// e^-9 of the first).
static ld gamma_moment(int m, double tau, double delta) {
    const ld t = tau, dl = delta, u = t * dl;
    if (u <= 3.0L) {
        // delta^(m+1) sum_i (-u^2)^i / (i! (m + 1 + 2i))
        ld term = 1.0L, sum = 0.0L;
        const ld u2 = u * u;
        for (int i = 0; i < 80; ++i) {
            sum += term / (m + 1 + 2 * i);
            term *= -u2 / (i + 1);
        }
        return powl(dl, m + 1) * sum;
    }
    const ld u2 = u * u, e = expl(-u2);
    const ld g12 = sqrtl(PI_L) * erfl(u);                 // gammainc(1/2, u^2)
    const ld g1 = -expm1l(-u2);                           // gammainc(1, u^2)
    const ld g32 = 0.5L * g12 - u * e;                    // gammainc(3/2, u^2)
    const ld g2 = g1 - u2 * e;                            // gammainc(2, u^2)
    const ld g52 = 1.5L * g32 - u2 * u * e;               // gammainc(5/2, u^2)
    ld g = 0.0L;
    switch (m) {
        case 1: g = g1; break;
        case 2: g = g32; break;
        case 3: g = g2; break;
        case 4: g = g52; break;
    }
    return g / (2.0L * powl(t, m + 1));
}

// int_0^delta r^m U(r) dr for the kernel (constants included)
static ld u_moment(int kernel, int m, double delta, double beta) {
    const ld dl = delta;
    switch (kernel) {
        case INVERSE_POWER: return powl(dl, m + 1 - (ld)beta) / (m + 1 - (ld)beta);
        case COULOMB_3D:
        case DIPOLAR_3D: return powl(dl, m) / (4.0L * PI_L * m);
        case COULOMB_2D: return powl(dl, m) / (2.0L * PI_L * m);
        case POISSON_2D:
        case DAVEY_STEWARTSON_2D: {
            const ld a = m + 1;
            return -powl(dl, a) * (logl(dl) / a - 1.0L / (a * a)) / (2.0L * PI_L);
        }
    }
    return 0.0L;
}

void taylor_constants(int kernel, int d, const Table& t, double& A0, double& c2) {
    if (kernel == GAUSSIAN_SUM) {
        A0 = c2 = 0.0;
        return;
    }
    const ld area = (d == 3) ? 4.0L * PI_L : 2.0L * PI_L;
    const int m0 = d - 1, m2 = d + 1;
    ld s0 = u_moment(kernel, m0, t.delta, t.beta), s2 = u_moment(kernel, m2, t.delta, t.beta);
    for (size_t q = 0; q < t.w.size(); ++q) {
        s0 -= (ld)t.w[q] * gamma_moment(m0, t.tau[q], t.delta);
        s2 -= (ld)t.w[q] * gamma_moment(m2, t.tau[q], t.delta);
    }
    A0 = (double)(area * s0);
    c2 = (double)(area * s2 / (2.0L * d));
}

// ------------------------------------------------------------------ host assembly

void assemble_spectrum(int d, const int* nk, const double* Lk, const Table& t, const std::vector<double>* Fk,
                       double A0, double c2, bool dxx, int lapu, std::vector<double>& S) {
    // Laplacian weights at indices all divisible by lapu / elsewhere (lapu = 0: 1 everywhere)
    const double lwe = lapu ? std::pow((double)lapu, d) : 1.0, lwo = lapu ? 0.0 : 1.0;
    const int lu = lapu ? lapu : 1;
    const int na = nk[0] + 1, nb = nk[1] + 1, nc = nk[d - 1] + 1, Q = (int)t.w.size();
    const double dxa = PI / (2.0 * Lk[0]), dxb = PI / (2.0 * Lk[1]), dxc = PI / (2.0 * Lk[d - 1]);
    const std::vector<double>& Fa = Fk[0];
    const std::vector<double>& Fb = Fk[1];
    const std::vector<double>& Fc = Fk[d - 1];
    double M = 1.0;
    for (int j = 0; j < d; ++j) M *= 2.0 * nk[j];
    const double invM = 1.0 / M;
    S.assign(d == 3 ? (size_t)na * nb * nc : (size_t)na * nb, 0.0);
    parallel_for(na, [&](int a0, int a1) {
        std::vector<double> wa(Q);
        for (int a = a0; a < a1; ++a) {
            for (int q = 0; q < Q; ++q) wa[q] = t.w[q] * Fa[(size_t)a * Q + q];
            const double xa = a * dxa;
            const double fa = dxx ? -(xa * xa) * invM : invM;
            if (d == 2) {
                for (int b = 0; b < nb; ++b) {
                    double acc = 0.0;
                    for (int q = 0; q < Q; ++q) acc += wa[q] * Fb[(size_t)b * Q + q];
                    const double xb = b * dxb;
                    const double lw = (a % lu == 0 && b % lu == 0) ? lwe : lwo;
                    S[(size_t)a * nb + b] = (acc + A0 - c2 * lw * (xa * xa + xb * xb)) * fa;
                }
                continue;
            }
            for (int b = 0; b < nb; ++b) {
                const double xb = b * dxb;
                for (int cc = 0; cc < nc; ++cc) {
                    double acc = 0.0;
                    for (int q = 0; q < Q; ++q) acc += wa[q] * Fb[(size_t)b * Q + q] * Fc[(size_t)cc * Q + q];
                    const double xc = cc * dxc;
                    const double lw = (a % lu == 0 && b % lu == 0 && cc % lu == 0) ? lwe : lwo;
                    S[((size_t)a * nb + b) * nc + cc] = (acc + A0 - c2 * lw * (xa * xa + xb * xb + xc * xc)) * fa;
                }
            }
        }
    });
}

void twiddles(int n, std::vector<double>& tw) {
    tw.resize(4 * (size_t)n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int m = 0; m < 2 * n; ++m) {
        const long double a = pi * (long double)m / (long double)n;
        tw[2 * m] = (double)cosl(a);
        tw[2 * m + 1] = (double)(-sinl(a));
    }
}

}  // namespace gsh
