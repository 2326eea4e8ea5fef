"""Pins of the oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check uses printed values of
the paper (tests/golden), closed-form potentials, an independent quadrature,
brute-force transforms, or an invariant of the continuous problem.
"""

import csv
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
import workloads
from oracle import closed_forms as cf
from oracle import dft, gs_table
from oracle.factors import factor_1d
from oracle.evaluate import full_spectrum, laplacian_symbol, periodic_laplacian
from oracle.taylor import taylor_constants


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(line for line in f if not line.startswith("#")))


def _exact(kernel, n, L, sigma, x0):
    d = 3 if kernel.endswith("3d") else 2
    X = workloads.mesh(n, L, d)
    if kernel == "dipolar3d":
        return cf.dipolar3d_gaussian(X[0], X[1], X[2], workloads.PAPER_DIPOLE_N,
                                     workloads.PAPER_DIPOLE_M, sigma)
    if kernel == "davey_stewartson2d":
        return cf.davey_stewartson_gaussian(*np.broadcast_arrays(X[0] - x0[0], X[1] - x0[1]))
    r = np.sqrt(sum((X[i] - x0[i]) ** 2 for i in range(d)))
    return {"coulomb3d": cf.coulomb3d_gaussian, "coulomb2d": cf.coulomb2d_gaussian,
            "poisson2d": cf.poisson2d_gaussian}[kernel](r, sigma)


# ---------------------------------------------------------------- paper tables

def _golden_error_rows():
    here = os.path.join(os.path.dirname(__file__), "golden", "paper_table_errors.csv")
    return _rows(here)


@pytest.mark.parametrize("row", _golden_error_rows(), ids=lambda r: f"{r['kernel']}-L{r['L']}-n{r['n']}")
def test_paper_table_error(row):
    kernel, L, n, sigma = row["kernel"], float(row["L"]), int(row["n"]), float(row["sigma"])
    d = 3 if kernel.endswith("3d") else 2
    x0 = [float(row["x0"]), float(row["y0"]), float(row["z0"])][:d]
    eps = 1e-13 if kernel in ("poisson2d", "davey_stewartson2d") else 1e-14
    dip = (workloads.PAPER_DIPOLE_N, workloads.PAPER_DIPOLE_M) if kernel == "dipolar3d" else None
    plan = oracle.make_plan(kernel, d, n, L, eps=eps, dipole=dip)
    scale = math.pi if kernel == "davey_stewartson2d" else 1.0
    rho = workloads.gaussian(n, L, d, sigma=sigma, center=x0, scale=scale)
    E = relmax(oracle.evaluate(plan, rho), _exact(kernel, n, L, sigma, x0))
    Ep = float(row["E_paper"])
    if row["check"] == "rel":
        assert abs(E - Ep) <= 0.01 * Ep, (E, Ep)
    elif row["check"] == "rel5":
        assert abs(E - Ep) <= 0.05 * Ep, (E, Ep)
    elif row["check"] == "le":
        assert E <= max(3 * Ep, 3e-15), (E, Ep)
    else:
        assert Ep / 10 <= E <= Ep * 10, (E, Ep)


def test_paper_max_norms(golden_dir):
    """Tables 3 and 5 print max|u|; the closed forms must reproduce them."""
    for row in _rows(os.path.join(golden_dir, "paper_max_norms.csv")):
        s, g, um = float(row["sigma"]), float(row["gamma"]), float(row["umax"])
        v = cf.anisotropic3d_max(s, g) if row["kernel"] == "coulomb3d" else cf.anisotropic2d_max(s, g)
        digits = len(row["umax"].replace("0.", "").replace(".", "").lstrip("0"))
        assert abs(v - um) <= 0.6 * 10 ** (math.floor(math.log10(um)) - digits + 1), (row, v)


def test_anisotropic_oracle_max_norm():
    """Table 3, gamma = 1: the oracle's max|u| on [-12,12]^3 equals sigma^2/2 = 2."""
    n, L = 48, 12.0
    plan = oracle.make_plan("coulomb3d", 3, n, L)
    u = oracle.evaluate(plan, workloads.gaussian(n, L, 3, sigma=2.0))
    assert abs(np.max(np.abs(u)) - 2.0) < 1e-8


def test_triaxial_closed_form_against_mpmath():
    a = (1.0, 4.0, 16.0)
    pts = [(0.0, 0.0, 0.0), (0.3, -0.7, 0.2), (2.0, 1.0, -1.5), (7.0, -3.0, 9.0)]
    for p in pts:
        v = cf.coulomb3d_triaxial(*[np.array([c]) for c in p], a=a)[0]
        assert abs(v - cf.coulomb3d_triaxial_mp(*p, a=a)) < 1e-14 * max(1.0, abs(v))
    # the isotropic case reduces to the erf form
    r = math.sqrt(0.3 ** 2 + 0.7 ** 2 + 0.2 ** 2)
    v = cf.coulomb3d_triaxial(np.array([0.3]), np.array([-0.7]), np.array([0.2]), a=(1, 1, 1))[0]
    assert abs(v - cf.coulomb3d_gaussian(np.array([r]), 1.0)[0]) < 1e-14


# ---------------------------------------------------------------- GS tables

def test_coulomb_table_meets_eps_off_grid():
    for d, dl in ((3, 1e-4), (2, 1e-3)):
        w, tau, S = gs_table.coulomb_table(d, dl, 1e-14)
        rng = np.random.default_rng(1)
        r = np.exp(rng.uniform(math.log(dl), math.log(2 * math.sqrt(d)), 20000))
        approx = np.sum(w[None, :] * np.exp(-(tau[None, :] * r[:, None]) ** 2), axis=1)
        assert np.max(np.abs(1.0 - r * approx)) < 2e-14
        assert len(w) == S + 1 and tau[0] == 0.0


def test_coulomb_table_convergence_rate():
    """Prop. 1: once the nodes cover the interval the error falls at least like
    exp(-C S / ln S); and the chosen S is the smallest one meeting eps."""
    Ss = (160, 200, 240)
    errs = [gs_table.coulomb_error(S, 1e-4, 2 * math.sqrt(3)) for S in Ss]
    x = [S / math.log(S) for S in Ss]
    for i in range(2):
        assert math.log(errs[i] / errs[i + 1]) / (x[i + 1] - x[i]) > 1.0, errs
    w, tau, S = gs_table.coulomb_table(3, 1e-4, 1e-14)
    assert gs_table.coulomb_error(S, 1e-4, 2 * math.sqrt(3)) <= 1e-14
    assert gs_table.coulomb_error(S - 1, 1e-4, 2 * math.sqrt(3)) > 1e-14


def test_poisson_table_meets_eps():
    dl, eps = 1e-3, 1e-13
    C0, wh, s, S = gs_table.poisson_table(dl, eps)
    X = 2 * math.sqrt(2) / dl
    rng = np.random.default_rng(2)
    x = np.exp(rng.uniform(0.0, math.log(X), 20000))
    approx = C0 - np.sum(wh[None, :] * np.exp(-s[None, :] * x[:, None] ** 2), axis=1)
    assert np.max(np.abs(np.log(x) - approx)) < 2 * eps


def test_physical_tables_reproduce_kernels():
    rng = np.random.default_rng(3)
    for kernel, d, eps in (("coulomb3d", 3, 1e-14), ("coulomb2d", 2, 1e-14), ("poisson2d", 2, 1e-13)):
        L = 7.0
        t = gs_table.physical_table(kernel, d, L, eps)
        r = np.exp(rng.uniform(math.log(t.delta), math.log(2 * math.sqrt(d) * L), 5000))
        ugs = np.sum(t.w[None, :] * np.exp(-(t.tau[None, :] * r[:, None]) ** 2), axis=1)
        if kernel == "coulomb3d":
            ex = 1 / (4 * math.pi * r)
            assert np.max(np.abs(ugs / ex - 1)) < 2e-14
        elif kernel == "coulomb2d":
            ex = 1 / (2 * math.pi * r)
            assert np.max(np.abs(ugs / ex - 1)) < 2e-14
        else:
            ex = -np.log(r) / (2 * math.pi)
            assert np.max(np.abs(ugs - ex)) < 3 * eps / (2 * math.pi) + 1e-15 * np.max(np.abs(ex))


# ---------------------------------------------------------------- 1-D factors

@pytest.mark.parametrize("L,n", [(8.0, 32), (10.0, 256)])
def test_factors_against_erf_closed_form(L, n):
    c = 2 * L
    taus = np.array([0.0, 1e-4, 0.003, 0.02, 0.1, 0.3, 0.6 / L * 5, 6.4 / c, 6.6 / c, 5.0, 300.0])
    F = factor_1d(taus, c, n)
    ks = sorted({0, 1, 2, 7, n // 3, n // 2, n - 1, n})
    for q, t in enumerate(taus):
        for k in ks:
            ref = cf.factor_mp(float(t), c, k)
            assert abs(F[k, q] - ref) <= 4e-16 * 2 * c, (t, k, F[k, q], ref)


def test_factor_special_values():
    c, n = 16.0, 64
    F = factor_1d(np.array([0.0, 0.05, 2.0]), c, n)
    assert F[0, 0] == 2 * c and np.all(F[1:, 0] == 0.0)
    assert abs(F[0, 1] - math.sqrt(math.pi) * math.erf(0.05 * c) / 0.05) < 1e-15 * 2 * c
    xi = math.pi * np.arange(n + 1) / c
    assert np.allclose(F[:, 2], math.sqrt(math.pi) / 2.0 * np.exp(-xi ** 2 / 16.0), rtol=0, atol=1e-18)


# ---------------------------------------------------------------- Taylor constants

def _u_of(kernel, r):
    if kernel == "coulomb3d":
        return 1 / (4 * mp.pi * r)
    if kernel == "coulomb2d":
        return 1 / (2 * mp.pi * r)
    return -mp.log(r) / (2 * mp.pi)


@pytest.mark.parametrize("kernel,d", [("coulomb3d", 3), ("coulomb2d", 2), ("poisson2d", 2)])
def test_taylor_constants_against_quadrature(kernel, d):
    """A0, c2 against a direct quadrature of int_0^delta r^m (U - U_GS) dr."""
    t = gs_table.physical_table(kernel, d, 9.0, 1e-13, delta_rel=1e-3)
    A0, c2 = taylor_constants(kernel, d, t.delta, t.w, t.tau)
    with mp.workdps(30):
        area = 2 * mp.pi ** (mp.mpf(d) / 2) / mp.gamma(mp.mpf(d) / 2)
        ws = [mp.mpf(float(x)) for x in t.w]
        ts = [mp.mpf(float(x)) for x in t.tau]

        def diff(r):
            return _u_of(kernel, r) - mp.fsum(wq * mp.exp(-(tq * r) ** 2) for wq, tq in zip(ws, ts))
        pts = [0] + [t.delta * 10 ** (-k) for k in range(8, 0, -1)] + [t.delta]
        q0 = area * mp.quad(lambda r: r ** (d - 1) * diff(r), pts)
        q2 = area * mp.quad(lambda r: r ** (d + 1) * diff(r), pts) / (2 * d)
    assert abs(A0 - float(q0)) <= 1e-12 * abs(float(q0))
    assert abs(c2 - float(q2)) <= 1e-12 * abs(float(q2))


def test_taylor_correction_exact_for_cubic_density():
    """For a cubic polynomial density the ball integral of (U - U_GS) rho(x - y)
    equals A0 rho(x) + c2 Lap rho(x) exactly (odd and mixed terms vanish)."""
    kernel, d = "coulomb3d", 3
    t = gs_table.physical_table(kernel, d, 1.0, 1e-12, delta_rel=0.05)
    A0, c2 = taylor_constants(kernel, d, t.delta, t.w, t.tau)
    dl = t.delta
    # rho(z) = 1 + 2 z1 - z2^2 + 3 z1 z3 + z3^2 + z1^3, at x = 0: rho = 1, Lap = 0 (-2 + 2)+6 z1 = 0
    # use rho(z) = 1 + z1 + 2 z1^2 + z2^2 - z3^2/2 + z1 z2 + z2^3: Lap(0) = 4 + 2 - 1 = 5
    with mp.workdps(25):
        ws = [mp.mpf(float(x)) for x in t.w]
        ts = [mp.mpf(float(x)) for x in t.tau]

        def radial(r):
            return 1 / (4 * mp.pi * r) - mp.fsum(wq * mp.exp(-(tq * r) ** 2) for wq, tq in zip(ws, ts))

        def rho_m(y1, y2, y3):      # rho(x - y) at x = 0
            z1, z2, z3 = -y1, -y2, -y3
            return 1 + z1 + 2 * z1 ** 2 + z2 ** 2 - z3 ** 2 / 2 + z1 * z2 + z2 ** 3

        # angular average of rho(-r omega) for the polynomial: 1 + r^2 (2 + 1 - 1/2)/3
        def integrand(r):
            ang = 4 * mp.pi * (1 + r * r * (mp.mpf(2) + 1 - mp.mpf(1) / 2) / 3)
            return r * r * radial(r) * ang
        val = mp.quad(integrand, [0, dl * 1e-6, dl * 1e-3, dl])
    assert abs(float(val) - (A0 * 1.0 + c2 * 5.0)) <= 1e-12 * abs(float(val))


# ---------------------------------------------------------------- transforms

def test_separable_dft_equals_full_dft():
    rng = np.random.default_rng(4)
    for shape in ((4, 4, 4), (6, 6), (5, 5, 5)):
        x = rng.standard_normal(shape)
        assert relmax(dft.forward(x), dft.full_dft(x)) < 1e-13
        assert relmax(dft.forward(x, sign=+1), dft.full_dft(x, sign=+1)) < 1e-13


def test_operator_is_aperiodic_toeplitz_convolution():
    """u_i = sum_j K[i - j] rho_j with K from the inverse transform of the
    spectrum: no wrap-around, independent of the grid origin."""
    rng = np.random.default_rng(5)
    for kernel, d, n in (("coulomb2d", 2, 6), ("coulomb3d", 3, 4), ("poisson2d", 2, 5)):
        L = 3.0
        plan = oracle.make_plan(kernel, d, n, L, eps=1e-13)
        M = plan.M
        Shat = oracle.full_spectrum(plan) + plan.A0 - plan.c2 * oracle.laplacian_symbol(plan)
        # K[m] for m in Z_{2n}^d from a plain full inverse DFT of the spectrum
        K = np.real(np.fft.ifftn(Shat)) * (M / M)   # numpy's ifftn divides by M already
        rho = rng.standard_normal((n,) * d)
        u = np.zeros_like(rho)
        idx = list(np.ndindex(*rho.shape))
        for i in idx:
            s = 0.0
            for j in idx:
                m = tuple((a - b) % (2 * n) for a, b in zip(i, j))
                s += K[m] * rho[j]
            u[i] = s
        assert relmax(oracle.evaluate(plan, rho), u) < 1e-12


def test_linearity_reversal_permutation_translation():
    rng = np.random.default_rng(6)
    n, L = 16, 4.0
    plan = oracle.make_plan("coulomb3d", 3, n, L)
    a = rng.standard_normal((n, n, n))
    b = rng.standard_normal((n, n, n))
    ua, ub = oracle.evaluate(plan, a), oracle.evaluate(plan, b)
    assert relmax(oracle.evaluate(plan, 2 * a - 3 * b), 2 * ua - 3 * ub) < 1e-13
    assert relmax(oracle.evaluate(plan, a[::-1, :, ::-1].copy()), ua[::-1, :, ::-1]) < 1e-13
    assert relmax(oracle.evaluate(plan, np.transpose(a, (2, 0, 1)).copy()), np.transpose(ua, (2, 0, 1))) < 1e-13
    # translation by 3 points along y of a density supported away from the edge
    c = np.zeros((n, n, n))
    c[3:9, 2:8, 4:12] = rng.standard_normal((6, 6, 8))
    cs = np.roll(c, 3, axis=1)
    u_c, u_cs = oracle.evaluate(plan, c), oracle.evaluate(plan, cs)
    assert relmax(u_cs[:, 3:, :], u_c[:, :-3, :]) < 1e-13


@pytest.mark.parametrize("kernel,d", [("coulomb3d", 3), ("coulomb2d", 2), ("poisson2d", 2)])
def test_box_scaling_covariance(kernel, d):
    """u_{sL}(s x) = s^{d-1} u_L(x) for Coulomb; s^2 [u_L(x) - ln(s)/(2pi) int rho] for Poisson."""
    rng = np.random.default_rng(7)
    n, L, s = 12, 3.0, 2.0
    rho = rng.standard_normal((n,) * d)
    eps = 1e-13 if kernel == "poisson2d" else 1e-14
    u1 = oracle.evaluate(oracle.make_plan(kernel, d, n, L, eps=eps), rho)
    u2 = oracle.evaluate(oracle.make_plan(kernel, d, n, s * L, eps=eps), rho)
    if kernel == "poisson2d":
        h = 2 * L / n
        ref = s ** 2 * (u1 - math.log(s) / (2 * math.pi) * h ** 2 * rho.sum())
    else:
        ref = s ** (d - 1) * u1
    assert relmax(u2, ref) < 1e-13


def test_tau_zero_term_is_a_constant():
    n, L, w0 = 10, 2.5, 0.37
    rng = np.random.default_rng(8)
    rho = rng.standard_normal((n, n))
    plan = oracle.make_plan("gaussian_sum", 2, n, L, custom=([w0], [0.0]))
    u = oracle.evaluate(plan, rho)
    h = 2 * L / n
    assert np.max(np.abs(u - w0 * h * h * rho.sum())) < 1e-14 * abs(w0 * h * h * rho.sum()) + 1e-15


def test_single_gaussian_kernel_gives_textbook_convolution():
    """U = exp(-tau^2 r^2) (no Taylor term) applied to exp(-a|x|^2): the product of
    the one-dimensional Gaussian convolutions sqrt(pi/(tau^2+a)) exp(-tau^2 a x^2/(tau^2+a))."""
    n, L, tau, a = 48, 6.0, 1.3, 2.0
    plan = oracle.make_plan("gaussian_sum", 3, n, L, custom=([1.0], [tau]))
    rho = workloads.gaussian(n, L, 3, sigma=1 / math.sqrt(a))
    X = workloads.mesh(n, L, 3)
    ex = 1.0
    for xi in X:
        ex = ex * math.sqrt(math.pi / (tau * tau + a)) * np.exp(-tau * tau * a * xi * xi / (tau * tau + a))
    assert relmax(oracle.evaluate(plan, rho), ex) < 1e-14


def test_spectral_laplacian_accuracy():
    n, L, sg = 64, 8.0, 1.5
    plan = oracle.make_plan("gaussian_sum", 3, n, L, custom=([0.0], [1.0]))
    rho = workloads.gaussian(n, L, 3, sigma=sg)
    lap = dft.inverse(-oracle.laplacian_symbol(plan) * dft.forward(rho)).real / plan.M
    X = workloads.mesh(n, L, 3)
    r2 = sum(x * x for x in X)
    ex = (4 * r2 / sg ** 4 - 6 / sg ** 2) * np.exp(-r2 / sg ** 2)
    # spectral differentiation amplifies rounding by |xi|_max^2 ~ 500 here
    assert relmax(lap, ex) < 1e-10


def test_each_taylor_term_is_needed():
    """With delta = 1e-3 L both correction terms are visible: dropping c2 Lap rho
    leaves ~1e-12, dropping A0 rho as well ~1e-6; with both the error is at roundoff."""
    n, L, sg = 64, 8.0, 1.2
    rho = workloads.gaussian(n, L, 3, sigma=sg)
    X = workloads.mesh(n, L, 3)
    ex = cf.coulomb3d_gaussian(np.sqrt(sum(x * x for x in X)), sg)
    plan = oracle.make_plan("coulomb3d", 3, n, L, eps=1e-14, delta_rel=1e-3)
    e_full = relmax(oracle.evaluate(plan, rho), ex)
    plan.c2 = 0.0
    e_noc2 = relmax(oracle.evaluate(plan, rho), ex)
    plan.A0 = 0.0
    e_none = relmax(oracle.evaluate(plan, rho), ex)
    assert e_full < 2e-15 and e_noc2 > 1e-13 and e_none > 1e-7, (e_full, e_noc2, e_none)


# ---------------------------------------------------------------- adjoint / energy

@pytest.mark.parametrize("kernel,d", [("coulomb3d", 3), ("poisson2d", 2), ("dipolar3d", 3)])
def test_adjoint_dot_and_symmetry(kernel, d):
    rng = np.random.default_rng(9)
    n, L = 10, 3.0
    dip = ((0.6, 0.8, 0.0), (0.0, 0.6, 0.8)) if kernel == "dipolar3d" else None
    plan = oracle.make_plan(kernel, d, n, L, eps=1e-13, dipole=dip)
    r, v = rng.standard_normal((2,) + (n,) * d)
    Ar, Atv = oracle.evaluate(plan, r), oracle.adjoint(plan, v)
    lhs, rhs = float(np.sum(Ar * v)), float(np.sum(r * Atv))
    assert abs(lhs - rhs) <= 1e-14 * np.sqrt(np.sum(Ar ** 2) * np.sum(v ** 2))
    assert relmax(Atv, oracle.evaluate(plan, v)) < 1e-13      # the kernel is even


def test_mixture_energy_matches_closed_form():
    rng = np.random.default_rng(10)
    mix = workloads.draw_mixture(rng, 4, 3, mu_range=1.5, sigma_range=(1.0, 1.6))
    n, L = 64, 10.0
    plan = oracle.make_plan("coulomb3d", 3, n, L)
    rho = workloads.sample_mixture(mix, n, L)
    E = oracle.energy(plan, rho)
    Eex = cf.mixture_energy_coulomb3d(mix.a, mix.mu, mix.sigma)
    assert abs(E - Eex) < 1e-9 * abs(Eex)


def test_coulomb_energy_is_positive():
    rng = np.random.default_rng(11)
    n, L = 16, 4.0
    plan = oracle.make_plan("coulomb3d", 3, n, L)
    for _ in range(3):
        rho = rng.standard_normal((n, n, n))
        assert oracle.energy(plan, rho) > 0.0


def test_dipolar_seeded_vectors_against_closed_form():
    p = workloads.config3_dipolar(n=64)
    plan = oracle.make_plan("dipolar3d", 3, p.n, p.L, dipole=(p.extra["n"], p.extra["m"]))
    X = workloads.mesh(p.n, p.L, 3)
    ex = cf.dipolar3d_gaussian(X[0], X[1], X[2], p.extra["n"], p.extra["m"], 1.2)
    assert relmax(oracle.evaluate(plan, p.rho), ex) < 1e-13


def test_dipolar_closed_form_against_mpmath_hessian():
    """The dipolar closed form (series near 0, Hessian formula elsewhere) against a
    high-precision numerical Hessian of the erf potential."""
    nv, mv, sg = (0.6, 0.8, 0.0), (0.0, 0.6, 0.8), 1.2
    with mp.workdps(40):
        s = mp.mpf(sg)

        def phi(a, b, c):
            r = mp.sqrt(a * a + b * b + c * c)
            return s ** 3 * mp.sqrt(mp.pi) * mp.erf(r / s) / (4 * r)
        for r in (0.1, 0.359, 0.361, 1.0, 3.0):
            x = [mp.mpf(r) / mp.sqrt(3)] * 3
            x[1] = -x[1]
            H = [[mp.diff(phi, tuple(x), tuple(int(k == i) + int(k == j) for k in range(3)))
                  for j in range(3)] for i in range(3)]
            nm = sum(a * b for a, b in zip(nv, mv))
            ref = -nm * mp.exp(-(r * r) / s ** 2) - 3 * sum(nv[i] * H[i][j] * mv[j] for i in range(3) for j in range(3))
            v = cf.dipolar3d_gaussian(np.array([float(x[0])]), np.array([float(x[1])]),
                                      np.array([float(x[2])]), nv, mv, sg)[0]
            assert abs(v - float(ref)) < 1e-13, (r, v, float(ref))
    # u(0) = 0: D(0) = -I/3
    z = cf.dipolar3d_gaussian(np.zeros(1), np.zeros(1), np.zeros(1), nv, mv, 1.2)
    assert abs(z[0]) < 1e-15


# ------------------------------------------------------------ parameter gradients

def _concat_grad(ga, gmu, gs):
    return np.concatenate([np.ravel(ga), np.ravel(gmu), np.ravel(gs)])


def test_mixture_parameter_gradient_matches_closed_form_energy():
    """On a resolving grid the discrete energy is the continuum mixture energy (closed
    form: pairwise erf interactions), so the chain-rule gradient must match a central
    difference of the closed form in every amplitude, centre and width."""
    m = workloads.config5_mixture()
    pl = oracle.make_plan("coulomb3d", 3, 64, 10.0)
    E, ga, gmu, gs = oracle.energy_gradient_params(pl, m.a, m.mu, m.sigma)
    Ec = oracle.closed_forms.mixture_energy_coulomb3d(m.a, m.mu, m.sigma)
    assert abs(E - Ec) <= 1e-10 * abs(Ec)
    hh = 1e-6

    def fd(f, x):
        out = np.zeros_like(x)
        for idx in np.ndindex(x.shape):
            xp, xm = x.copy(), x.copy()
            xp[idx] += hh
            xm[idx] -= hh
            out[idx] = (f(xp) - f(xm)) / (2 * hh)
        return out

    cf = oracle.closed_forms.mixture_energy_coulomb3d
    ref = _concat_grad(fd(lambda v: cf(v, m.mu, m.sigma), m.a), fd(lambda v: cf(m.a, v, m.sigma), m.mu),
                       fd(lambda v: cf(m.a, m.mu, v), m.sigma))
    got = _concat_grad(ga, gmu, gs)
    assert np.max(np.abs(got - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_mixture_parameter_gradient_matches_discrete_difference():
    """On an under-resolved grid (no closed form) the chain rule must still be the
    derivative of the discrete energy: central differences of oracle energies."""
    rng = np.random.default_rng(3)
    mix = workloads.draw_mixture(rng, 3, 3)
    pl = oracle.make_plan("coulomb3d", 3, 12, 4.0)
    _, ga, gmu, gs = oracle.energy_gradient_params(pl, mix.a, mix.mu, mix.sigma)

    def E(a, mu, s):
        rho, _ = oracle.mixture_grid(12, 4.0, a, mu, s)
        return oracle.energy(pl, rho)

    hh = 1e-5
    got = _concat_grad(ga, gmu, gs)
    ref = []
    for which, x in (("a", mix.a), ("mu", mix.mu), ("s", mix.sigma)):
        for idx in np.ndindex(x.shape):
            args = {"a": mix.a.copy(), "mu": mix.mu.copy(), "s": mix.sigma.copy()}
            args[which][idx] += hh
            ep = E(args["a"], args["mu"], args["s"])
            args[which][idx] -= 2 * hh
            em = E(args["a"], args["mu"], args["s"])
            ref.append((ep - em) / (2 * hh))
    ref = np.array(ref)
    assert np.max(np.abs(got - ref)) <= 1e-7 * np.max(np.abs(ref))


# --------------------------------------------------------------------------
# Rectangular boxes (Section 2.5): one half-width per axis, n points per axis.
# --------------------------------------------------------------------------

def _rect_exact(p):
    X = workloads.mesh(p.n, p.L, p.d)
    s, g = p.extra["sigma"], p.extra["gamma"]
    if p.d == 3:
        x, y, z = np.broadcast_arrays(*X)
        return cf.coulomb3d_triaxial(x, y, z, a=(1 / s ** 2, 1 / s ** 2, g * g / s ** 2)).reshape(p.rho.shape)
    x, y = np.broadcast_arrays(X[0], X[1])
    return cf.coulomb2d_anisotropic(x, y, s, g).reshape(p.rho.shape)


@pytest.mark.parametrize("d,gamma,n", [(3, 2.0, 48), (3, 8.0, 48), (2, 4.0, 96), (2, 16.0, 96)])
def test_rectangular_box_against_closed_form(d, gamma, n):
    """Tables 3 and 5 setups (sigma = 2, box [-12,12]^(d-1) x [-12,12]/gamma): the
    oracle meets the closed-form potential of the anisotropic Gaussian at every
    grid point (the paper reports 5.6e-16 .. 2.6e-14 for these rows)."""
    p = workloads.rect_box(d, gamma, n=n)
    plan = oracle.make_plan(p.kernel, d, n, p.L)
    u = oracle.evaluate(plan, p.rho)
    assert relmax(u, _rect_exact(p)) < 1e-13


def test_rectangular_box_max_norms(golden_dir):
    """max|u| on the rectangular boxes reproduces the printed column of Tables 3 and 5."""
    for row in _rows(os.path.join(golden_dir, "paper_max_norms.csv")):
        d = 3 if row["kernel"] == "coulomb3d" else 2
        g = float(row["gamma"])
        if g == 1.0 or g == 16.0:
            continue
        p = workloads.rect_box(d, g, n=48 if d == 3 else 96)
        u = oracle.evaluate(oracle.make_plan(p.kernel, d, p.n, p.L), p.rho)
        um = float(row["umax"])
        digits = len(row["umax"].replace("0.", "").replace(".", "").lstrip("0"))
        assert abs(np.max(np.abs(u)) - um) <= 0.6 * 10 ** (math.floor(math.log10(um)) - digits + 1), row


def test_anisotropic_2d_closed_form_against_mpmath():
    for x, y, g in [(0.7, -0.3, 4.0), (0.0, 0.0, 16.0), (2.5, 0.4, 2.0), (-1.0, 1.5, 1.0)]:
        v = cf.coulomb2d_anisotropic(np.array([x]), np.array([y]), 2.0, g)[0]
        assert abs(v - cf.coulomb2d_anisotropic_mp(x, y, 2.0, g)) < 1e-14 * max(1.0, abs(v))
    # gamma = 1 is the isotropic Bessel form
    r = np.array([0.0, 0.8, 3.0])
    v = cf.coulomb2d_anisotropic(r, np.zeros(3), 1.5, 1.0)
    assert np.max(np.abs(v - cf.coulomb2d_gaussian(r, 1.5))) < 1e-14


@pytest.mark.parametrize("kernel,d,eps", [("coulomb3d", 3, 1e-14), ("poisson2d", 2, 1e-12)])
def test_rectangular_box_with_equal_sides_is_the_cube(kernel, d, eps):
    rng = np.random.default_rng(5)
    rho = rng.standard_normal((12,) * d)
    a = oracle.make_plan(kernel, d, 12, 5.0, eps=eps)
    b = oracle.make_plan(kernel, d, 12, (5.0,) * d, eps=eps)
    assert a.table.S == b.table.S and np.array_equal(a.G_oct, b.G_oct)
    assert np.array_equal(oracle.evaluate(a, rho), oracle.evaluate(b, rho))


@pytest.mark.parametrize("kernel", ["coulomb3d", "dipolar3d"])
def test_rectangular_box_axis_permutation(kernel):
    """Reversing the axes of box and density reverses the potential (with the
    dipole vectors' components permuted alike): a per-axis factor, frequency or
    Laplacian term attached to the wrong axis breaks it."""
    rng = np.random.default_rng(6)
    n = 16
    rho = rng.standard_normal((n,) * 3)
    dip = ((0.3, -0.5, 0.8), (0.6, 0.2, -0.4))
    a = oracle.make_plan(kernel, 3, n, (3.0, 4.0, 5.0), dipole=dip)
    rdip = (tuple(dip[0][::-1]), tuple(dip[1][::-1]))
    b = oracle.make_plan(kernel, 3, n, (5.0, 4.0, 3.0), dipole=rdip)
    ua = oracle.evaluate(a, rho)
    ub = oracle.evaluate(b, rho.transpose(2, 1, 0))
    assert relmax(ub.transpose(2, 1, 0), ua) < 1e-14


def test_rectangular_box_isotropic_gaussians():
    """An isotropic density in a rectangular box: 3D Coulomb and dipolar (per-axis
    frequencies in the dipolar symbol) and 2D Poisson against their closed forms."""
    n, Ls, s = 64, (7.0, 8.0, 9.0), 1.2
    rho = workloads.gaussian(n, Ls, 3, sigma=s)
    X = workloads.mesh(n, Ls, 3)
    r = np.sqrt(X[0] ** 2 + X[1] ** 2 + X[2] ** 2)
    u = oracle.evaluate(oracle.make_plan("coulomb3d", 3, n, Ls), rho)
    assert relmax(u, np.broadcast_to(cf.coulomb3d_gaussian(r, s), u.shape)) < 1e-13
    dn, dm = workloads.PAPER_DIPOLE_N, workloads.PAPER_DIPOLE_M
    u = oracle.evaluate(oracle.make_plan("dipolar3d", 3, n, Ls, dipole=(dn, dm)), rho)
    ex = cf.dipolar3d_gaussian(X[0], X[1], X[2], dn, dm, s)
    assert relmax(u, np.broadcast_to(ex, u.shape)) < 1e-12
    n2, L2 = 96, (9.0, 12.0)
    rho2 = workloads.gaussian(n2, L2, 2, sigma=s)
    Y = workloads.mesh(n2, L2, 2)
    r2 = np.sqrt(Y[0] ** 2 + Y[1] ** 2)
    u2 = oracle.evaluate(oracle.make_plan("poisson2d", 2, n2, L2, eps=1e-13), rho2)
    assert relmax(u2, np.broadcast_to(cf.poisson2d_gaussian(r2, s), u2.shape)) < 1e-13


def test_rectangular_box_table_and_near_field_rule():
    """The table is fitted on the distances of the box (R = 2 |L| / max L) and the
    near-field ball must fit the short axis (delta below eta)."""
    t = gs_table.physical_table("coulomb3d", 3, (1.5, 12.0, 12.0), 1e-14)
    hi = 2.0 * math.sqrt(2.0 + (1.5 / 12.0) ** 2)
    r = np.geomspace(1e-4, hi, 20001) * 12.0
    approx = sum(wq * np.exp(-(tq * r) ** 2) for wq, tq in zip(t.w, t.tau))
    assert np.max(np.abs(1.0 - 4.0 * math.pi * r * approx)) <= 1e-14
    with pytest.raises(ValueError):
        gs_table.physical_table("coulomb3d", 3, (1e-3, 12.0, 12.0), 1e-14, delta_rel=1e-4)


# --------------------------------------------------------------------------
# Davey-Stewartson potential (Example 4.5): Poisson kernel convolved with d_xx rho.
# --------------------------------------------------------------------------

def test_davey_stewartson_closed_form_against_mpmath():
    def direct(x, y):
        with mp.workdps(40):
            x, y = mp.mpf(x), mp.mpf(y)
            r2 = x * x + y * y
            if r2 == 0:
                return float(-mp.pi / 2)
            a = mp.pi ** 2 * r2
            return float(-(mp.pi / 2 * mp.e ** (-a)
                           + (x * x - y * y) / r2 * mp.e ** (-a) * (1 + a - mp.e ** a) / (2 * mp.pi * r2)))
    for x, y in [(0.0, 0.0), (0.05, 0.02), (0.1, 0.12), (0.3, -0.4), (0.7, 0.1), (1.2, 0.9), (3.0, 0.5), (-6.0, 2.0)]:
        v = cf.davey_stewartson_gaussian(np.array([x]), np.array([y]))[0]
        assert abs(v - direct(x, y)) <= 1e-15 * max(1.0, abs(v)), (x, y)


def test_davey_stewartson_xx_plus_yy_is_minus_rho():
    """d_xx + d_yy = Laplacian and -Laplacian of the Poisson kernel is the delta function:
    DS(rho) + (the same with x and y exchanged) = -rho, independently of the closed form
    (a wrong sign or axis of the symbol, or a lost Taylor term, breaks it)."""
    n, L = 128, 6.0
    rho = workloads.gaussian(n, L, 2, sigma=0.8, center=(0.3, -0.5)) - 0.5 * workloads.gaussian(n, L, 2, sigma=0.6)
    plan = oracle.make_plan("davey_stewartson2d", 2, n, L, eps=1e-13)
    uxx = oracle.evaluate(plan, rho)
    uyy = oracle.evaluate(plan, rho.T.copy()).T
    assert relmax(uxx + uyy, -rho) < 1e-12


def test_davey_stewartson_adjoint_and_symmetry():
    rng = np.random.default_rng(11)
    n = 16
    plan = oracle.make_plan("davey_stewartson2d", 2, n, 4.0, eps=1e-13)
    a, b = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    Aa, ATb = oracle.evaluate(plan, a), oracle.adjoint(plan, b)
    assert abs(np.sum(Aa * b) - np.sum(a * ATb)) <= 1e-13 * np.sqrt(np.sum(Aa ** 2) * np.sum(b ** 2))
    assert relmax(oracle.adjoint(plan, a), Aa) < 1e-13


# --------------------------------------------------------------------------
# Inverse-power kernels |x|^-beta (the Remark after eq. (GauInte)).
# --------------------------------------------------------------------------

@pytest.mark.parametrize("beta,d", [(0.5, 3), (2.0, 3), (2.5, 3), (1.5, 2)])
def test_power_closed_form_against_mpmath(beta, d):
    r = np.array([0.0, 0.3, 1.7, 5.0])
    v = cf.power_gaussian(r, beta, 1.3, d)
    for ri, vi in zip(r, v):
        assert abs(vi - cf.power_gaussian_mp(float(ri), beta, 1.3, d)) <= 1e-14 * abs(vi)
    assert abs(v[0] - cf.power_gaussian_origin(beta, 1.3, d)) <= 1e-14 * v[0]


@pytest.mark.parametrize("beta,d,n", [(0.5, 3, 48), (2.0, 3, 48), (2.5, 3, 48), (0.5, 2, 96), (1.5, 2, 96)])
def test_power_kernel_against_closed_form(beta, d, n):
    L, s = 8.0, 1.2
    rho = workloads.gaussian(n, L, d, sigma=s)
    X = np.broadcast_arrays(*workloads.mesh(n, L, d))
    r = np.sqrt(sum(x * x for x in X))
    u = oracle.evaluate(oracle.make_plan("inverse_power", d, n, L, beta=beta), rho)
    assert relmax(u, cf.power_gaussian(r, beta, s, d)) < 1e-13


@pytest.mark.parametrize("d,kernel,kappa", [(3, "coulomb3d", 4 * math.pi), (2, "coulomb2d", 2 * math.pi)])
def test_power_kernel_beta_one_is_coulomb(d, kernel, kappa):
    """beta = 1 is the Coulomb kernel without its constant, through a different table."""
    rng = np.random.default_rng(12)
    n = 16 if d == 3 else 48
    rho = rng.standard_normal((n,) * d)
    a = oracle.evaluate(oracle.make_plan("inverse_power", d, n, 5.0, beta=1.0), rho)
    b = oracle.evaluate(oracle.make_plan(kernel, d, n, 5.0), rho)
    assert relmax(a, kappa * b) < 1e-13


@pytest.mark.parametrize("beta,d", [(0.7, 3), (2.2, 3), (1.3, 2)])
def test_power_kernel_box_scaling(beta, d):
    """|s x|^-beta = s^-beta |x|^-beta: u_{sL}(s x) = s^(d - beta) u_L(x)."""
    rng = np.random.default_rng(13)
    n, L, s = 12, 3.0, 2.5
    rho = rng.standard_normal((n,) * d)
    u1 = oracle.evaluate(oracle.make_plan("inverse_power", d, n, L, beta=beta), rho)
    u2 = oracle.evaluate(oracle.make_plan("inverse_power", d, n, s * L, beta=beta), rho)
    assert relmax(u2, s ** (d - beta) * u1) < 1e-13


@pytest.mark.parametrize("beta,d", [(0.5, 3), (2.5, 3), (1.5, 2)])
def test_power_table_and_taylor_constants(beta, d):
    """The table meets eps on its fit interval; A0, c2 against a direct quadrature of
    int_0^delta r^m (r^-beta - U_GS) dr; beta outside (0, d) is refused."""
    hi = 2 * math.sqrt(d)
    w, tau, S = gs_table.power_table(beta, 1e-3, 1e-13, hi)
    assert gs_table.power_error(beta, S, 1e-3, hi, 1e-13) <= 1e-13
    t = gs_table.physical_table("inverse_power", d, 9.0, 1e-13, delta_rel=1e-3, beta=beta)
    A0, c2 = taylor_constants("inverse_power", d, t.delta, t.w, t.tau, beta)
    with mp.workdps(30):
        area = 2 * mp.pi ** (mp.mpf(d) / 2) / mp.gamma(mp.mpf(d) / 2)
        ws = [mp.mpf(float(x)) for x in t.w]
        ts = [mp.mpf(float(x)) for x in t.tau]

        def diff(r):
            return r ** (-mp.mpf(beta)) - mp.fsum(wq * mp.exp(-(tq * r) ** 2) for wq, tq in zip(ws, ts))
        pts = [0] + [t.delta * 10 ** (-k) for k in range(8, 0, -1)] + [t.delta]
        q0 = area * mp.quad(lambda r: r ** (d - 1) * diff(r), pts)
        q2 = area * mp.quad(lambda r: r ** (d + 1) * diff(r), pts) / (2 * d)
    assert abs(A0 - float(q0)) <= 1e-12 * abs(float(q0))
    assert abs(c2 - float(q2)) <= 1e-12 * abs(float(q2))
    with pytest.raises(ValueError):
        gs_table.physical_table("inverse_power", d, 9.0, 1e-13, beta=float(d))


# --------------------------------------------------------------------------
# Order of the near-field Taylor correction (Section 2.3, the bound after
# eq. (taylor)): with the Taylor constants of the ball |y| < delta, the
# remainder of the near-field integral is O(delta^(d+3)) for the Coulomb kernels
# and O(delta^6 |ln delta|) for the logarithmic one.
# --------------------------------------------------------------------------

_U_MP = {"coulomb3d": lambda r: 1 / (4 * mp.pi * r), "coulomb2d": lambda r: 1 / (2 * mp.pi * r),
         "poisson2d": lambda r: -mp.log(r) / (2 * mp.pi)}


def _near_field_remainder(kernel, d, delta, w, tau, x=0.7):
    """|N - (A0 rho(x) + c2 Lap rho(x))| for rho = exp(-|y|^2) at |x| = 0.7, where
    N = int_{|y|<delta} (U - U_GS)(|y|) rho(x - y) dy by mpmath quadrature over the
    radius of the exact spherical mean of the Gaussian (3D: e^{-(a^2+r^2)} sinh(2ar)/(2ar),
    2D: e^{-(a^2+r^2)} I0(2ar)); A0, c2 from the oracle for the table (w, tau)."""
    with mp.workdps(40):
        a = mp.mpf(x)

        def mean(r):
            z = 2 * a * r
            rad = mp.e ** (-(a * a + r * r))
            return rad * (mp.sinh(z) / z if d == 3 else mp.besseli(0, z))

        def ugs(r):
            return sum(mp.mpf(wq) * mp.e ** (-(mp.mpf(tq) * r) ** 2) for wq, tq in zip(w, tau))

        area = 4 * mp.pi if d == 3 else 2 * mp.pi
        N = area * mp.quad(lambda r: r ** (d - 1) * (_U_MP[kernel](r) - ugs(r)) * mean(r), [0, delta])
        A0, c2 = taylor_constants(kernel, d, delta, w, tau)
        rho = mp.e ** (-a * a)
        lap = rho * (4 * a * a - 2 * d)
        return float(abs(N - (A0 * rho + c2 * lap)))


@pytest.mark.parametrize("kernel,d", [("coulomb3d", 3), ("coulomb2d", 2), ("poisson2d", 2)])
@pytest.mark.parametrize("table", ["none", "two_terms"])
def test_taylor_remainder_delta_order(kernel, d, table):
    """Halving delta divides the remainder by 2^(d+3) (Coulomb) or by 2^6 up to the
    |ln delta| factor (ln kernel): a dropped or mis-scaled term of A0 or c2 leaves a
    remainder of order delta^(d-1) or delta^(d+1) and fails the slope.  With a Gaussian
    sum in the ball its smooth part only adds terms of higher order."""
    w, tau = ([], []) if table == "none" else ([0.3, -0.1], [0.0, 2.5])
    ds = [0.0125, 0.025, 0.05]
    e = np.array([_near_field_remainder(kernel, d, dl, w, tau) for dl in ds])
    if kernel == "poisson2d":
        # delta^6 (a |ln delta| + b): local slopes 6 + 1/ln delta, about 5.7 here
        slopes = np.diff(np.log(e)) / np.diff(np.log(ds))
        assert np.all((slopes > 5.3) & (slopes < 6.1)), slopes
        if table == "none":                    # the logarithmic factor itself
            ratio = e / np.array([dl ** 6 * abs(math.log(dl)) for dl in ds])
            assert np.max(ratio) / np.min(ratio) < 1.05, ratio
    else:
        slopes = np.diff(np.log(e)) / np.diff(np.log(ds))
        assert np.all(np.abs(slopes - (d + 3)) < 0.1), slopes


@pytest.mark.parametrize("tau", [1e-9, 1e-6, 1e-3, 0.004])
def test_factors_small_tau_relative_to_their_size(tau):
    """tau c <= 0.05 (the ln table's tiny exponents): the factors at k >= 1 are of the size
    (tau c)^2 c, far below 4L; mpmath quadrature over half-periods fixes them to 1e-15 of
    their own size, not only of 4L (the Davey-Stewartson symbol -xi_x^2 amplifies their
    absolute error)."""
    c, n = 12.0, 192
    F = factor_1d(np.array([tau]), c, n)[:, 0]
    with mp.workdps(40):
        for k in (0, 1, 2, 7, 50, n // 2, n):
            ex = mp.quad(lambda y: mp.e ** (-(tau * y) ** 2) * mp.cos(mp.pi * k * y / c),
                         mp.linspace(-c, c, 2 * max(k, 1) + 1))
            assert abs(F[k] - float(ex)) <= 1e-15 * abs(float(ex)), (k, F[k], ex)


# --------------------------------------------------------------------------
# Grids whose axes have their own n (Section 2.5: the box prod_j [-L_j, L_j] with
# n_j points on axis j; equal steps h on unequal sides need unequal n).
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kernel,n,L,sigma", [("coulomb3d", (64, 96, 128), (4.0, 6.0, 8.0), 0.6),
                                              ("coulomb3d", (96, 48, 64), (6.0, 3.0, 4.0), 0.45),
                                              ("poisson2d", (96, 192), (6.0, 12.0), 0.8),
                                              ("coulomb2d", (192, 64), (12.0, 4.0), 0.5)])
def test_per_axis_points_gaussian_closed_form(kernel, n, L, sigma):
    """A resolved Gaussian exp(-|x|^2/sigma^2) inside a box with unequal sides and the same
    step h = 1/8 on every axis (so unequal n_j): the potential matches the closed form to
    1e-13 of its maximum, as on cubes."""
    d = len(n)
    rho = workloads.gaussian(n, L, d, sigma=sigma)
    u = oracle.evaluate(oracle.make_plan(kernel, d, n, L, eps=1e-13 if kernel == "poisson2d" else 1e-14), rho)
    X = np.broadcast_arrays(*workloads.mesh(n, L, d))
    r = np.sqrt(sum(x * x for x in X))
    ex = {"coulomb3d": cf.coulomb3d_gaussian, "coulomb2d": cf.coulomb2d_gaussian,
          "poisson2d": cf.poisson2d_gaussian}[kernel](r, sigma)
    assert relmax(u, ex) <= 1e-13


def test_per_axis_points_axis_permutation():
    """Exchanging two axes (their n, L and the density's axes) exchanges the potential's
    axes: the per-axis n enters the factors, frequencies and padding of its own axis only."""
    rng = np.random.default_rng(17)
    n, L = (12, 20, 16), (3.0, 5.0, 4.0)
    rho = rng.standard_normal(n)
    u = oracle.evaluate(oracle.make_plan("coulomb3d", 3, n, L), rho)
    perm = (2, 0, 1)
    np_, Lp = tuple(n[i] for i in perm), tuple(L[i] for i in perm)
    up = oracle.evaluate(oracle.make_plan("coulomb3d", 3, np_, Lp), np.transpose(rho, perm))
    assert relmax(np.transpose(u, perm), up) <= 1e-14


# --------------------------------------------------------------------------
# The Taylor term's Laplacian on the density's own grid (Algorithm 1 step 3 read as the
# spectral Laplacian of the sampled density, period 2L), the fidelity variant of the
# Laplacian on the padded grid.
# --------------------------------------------------------------------------

def test_periodic_laplacian_exact_on_trigonometric_polynomials():
    """cos(pi k x / L) sin(pi m y / L) on the periodic n-point grid: Laplacian
    -(pi/L)^2 (k^2 + m^2) times itself, exactly up to rounding, for |k|, |m| < n/2 (and the
    Nyquist cosine k = n/2 with (pi/h)^2)."""
    n, L = (24, 16), (3.0, 2.0)
    plan = oracle.make_plan("coulomb2d", 2, n, L, laplacian="unpadded")
    X = np.broadcast_arrays(*workloads.mesh(n, L, 2))
    for kx, ky in [(1, 2), (5, 7), (7, 11), (8, 12)]:     # (8, 12): both Nyquist cosines
        f = np.cos(math.pi * kx * X[0] / L[1]) * np.cos(math.pi * ky * X[1] / L[0])
        want = -((math.pi * kx / L[1]) ** 2 + (math.pi * ky / L[0]) ** 2) * f
        assert np.max(np.abs(periodic_laplacian(plan, f) - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("kernel,d,n,L", [("coulomb3d", 3, 24, 5.0), ("poisson2d", 2, (32, 48), (4.0, 6.0)),
                                          ("dipolar3d", 3, 16, 4.0), ("davey_stewartson2d", 2, 24, 4.0)])
def test_unpadded_laplacian_variant(kernel, d, n, L):
    """The two readings differ only through c2 Lap rho: on a resolved Gaussian both match the
    closed form as closely (the correction is ~1e-17 at delta = 1e-4 L); on rough input
    they differ by exactly c2 (Lap_unpadded - Lap_padded) rho; the adjoint stays the
    transpose (dot test)."""
    kw = {"dipole": ((0.6, 0.8, 0.0), (0.0, 0.6, 0.8))} if kernel == "dipolar3d" else {}
    eps = 1e-13 if kernel in ("poisson2d", "davey_stewartson2d") else 1e-14
    pp = oracle.make_plan(kernel, d, n, L, eps=eps, **kw)
    pu = oracle.make_plan(kernel, d, n, L, eps=eps, laplacian="unpadded", **kw)
    rng = np.random.default_rng(31)
    ns = pp.ns
    x, v = rng.standard_normal(ns), rng.standard_normal(ns)
    up, uu = oracle.evaluate(pp, x), oracle.evaluate(pu, x)
    assert np.max(np.abs(uu - up)) > 0.0
    if kernel in ("coulomb3d", "poisson2d"):
        from oracle import dft
        lap_p = dft.inverse(-oracle.laplacian_symbol(pp) * dft.forward(x)).real / pp.M
        lap_u = periodic_laplacian(pu, x)
        assert np.max(np.abs((uu - up) - pp.c2 * (lap_u - lap_p))) <= 1e-14 * np.max(np.abs(up))
    lhs = float(np.sum(oracle.evaluate(pu, x) * v))
    rhs = float(np.sum(x * oracle.adjoint(pu, v)))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(uu) * np.linalg.norm(v)


# --------------------------------------------------------------------------
# Padding to B_3 (eq. (FourSeriB3) with n~ = 3n): transforms of length 3n, frequencies
# pi k / (3L), the factor integrals still over [-2L, 2L] (eq. (tensor)).
# --------------------------------------------------------------------------

@pytest.mark.parametrize("L,n", [(8.0, 32), (10.0, 128)])
def test_factors_padding3_against_erf_closed_form(L, n):
    """Factors at xi_k = 2 pi k / (3c), k = 0..3n/2, in every branch (tau = 0, the series,
    Gauss-Legendre, the closed form) against the erf closed form, to a few ulps of 2c."""
    c = 2 * L
    taus = np.array([0.0, 1e-7, 1e-4, 0.003, 0.02, 0.1, 0.3, 0.6 / L * 5, 6.4 / c, 6.6 / c, 5.0, 300.0])
    m = 3 * n // 2
    F = factor_1d(taus, c, m, 3)
    ks = sorted({0, 1, 2, 3, 7, n // 3, n // 2, n - 1, n, m - 1, m})
    for q, t in enumerate(taus):
        for k in ks:
            ref = cf.factor_mp(float(t), c, k, p=3)
            assert abs(F[k, q] - ref) <= 4e-16 * 2 * c, (t, k, F[k, q], ref)


def test_factor_mp_general_frequency_against_quadrature():
    """The closed form at frequencies that are not multiples of pi / c (mpmath quadrature)."""
    c = 3.0
    for tau, k in [(0.0, 1), (0.0, 5), (0.2, 1), (0.7, 4), (1.5, 7)]:
        xi = 2 * mp.pi * k / (3 * c)
        with mp.workdps(30):
            ref = mp.quad(lambda y: mp.exp(-(tau * y) ** 2) * mp.cos(xi * y), [-c, 0, c])
        assert abs(cf.factor_mp(tau, c, k, p=3) - float(ref)) <= 1e-15 * 2 * c


def _brute_force_potential(w, tau, A0, c2, n, L, rho, p):
    """The regular integral of eq. (I1FFT) with the trapezoidal coefficients of eq. (rho_hat)
    written out as one kernel matrix: u_i = sum_j K(x_i - x_j) rho_j with
    K(z) = (1/M) sum_k [sum_q w_q prod_j g_q(xi_kj) + A0 - c2 |xi_k|^2] exp(i xi_k . z),
    k over [-p n_j / 2, p n_j / 2)^d, xi_kj = pi k_j / (p L_j), g_q by the closed form,
    M = prod_j p n_j; no padding, transform or crop."""
    d = len(n)
    axes = []
    for nj, Lj in zip(n, L):
        ks = np.arange(-p * nj // 2, p * nj // 2)
        g = np.array([[cf.factor_mp(float(t), 2 * Lj, abs(int(k)), p=p) for t in tau] for k in ks])   # (K, Q)
        axes.append((ks, g, math.pi * ks / (p * Lj), 2 * Lj / nj))
    M = float(np.prod([p * nj for nj in n]))
    idx = list(np.ndindex(*n))
    u = np.zeros(n)
    # kernel values at every grid difference (C-order axes)
    Kval = {}
    for diff in np.ndindex(*[2 * nj - 1 for nj in n]):
        z = [(dj - (nj - 1)) * ax[3] for dj, nj, ax in zip(diff, n, axes)]
        tot = 0.0
        grids = np.meshgrid(*[np.arange(len(ax[0])) for ax in axes], indexing="ij")
        gk = np.zeros(grids[0].shape)
        for q in range(len(w)):
            term = w[q]
            for a, ax in enumerate(axes):
                term = term * ax[1][grids[a], q]
            gk = gk + term
        xis = [ax[2][grids[a]] for a, ax in enumerate(axes)]
        sym = gk + A0 - c2 * sum(x * x for x in xis)
        ph = sum(x * zj for x, zj in zip(xis, z))
        tot = float(np.sum(sym * np.cos(ph))) / M
        Kval[tuple(dj - (nj - 1) for dj, nj in zip(diff, n))] = tot
    for i in idx:
        s = 0.0
        for j in idx:
            s += Kval[tuple(a - b for a, b in zip(i, j))] * rho[j]
        u[i] = s
    return u


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("d,n,L", [(2, (6, 4), (1.5, 1.0)), (3, (4, 4, 2), (1.0, 1.0, 0.5))])
def test_padding_brute_force_convolution(p, d, n, L):
    """A Gaussian sum with terms in every factor branch (tau = 0, series, quadrature,
    closed form) plus Taylor-like constants: the oracle's padded transforms equal the
    kernel-matrix sum of the same coefficients (closed-form factors), for p = 2 and 3."""
    w = [0.37, -0.8, 1.3, 0.45, 2.0]
    tau = [0.0, 0.01, 0.45, 1.7, 9.0]
    rng = np.random.default_rng(40 + p + d)
    rho = rng.standard_normal(n)
    plan = oracle.make_plan("gaussian_sum", d, n, L, custom=(w, tau), padding=p)
    A0, c2 = 0.3, 0.02
    plan.A0, plan.c2 = A0, c2
    u = oracle.evaluate(plan, rho)
    ref = _brute_force_potential(w, tau, A0, c2, n, L, rho, p)
    assert relmax(u, ref) <= 1e-13


@pytest.mark.parametrize("kernel,d,n,L,sigma", [("coulomb3d", 3, 64, 8.0, 1.0),
                                                ("poisson2d", 2, 64, 8.0, 1.0),
                                                ("coulomb2d", 2, (48, 64), (6.0, 8.0), 0.8)])
def test_padding3_resolved_gaussian_closed_form(kernel, d, n, L, sigma):
    """A resolved Gaussian (h = 1/4): padding to B_3 reaches the closed form as closely as
    padding to B_2 (the readings differ through the interpolant's ripples between the
    samples, which the integral over two thirds of the period B_3 does not cancel)."""
    rho = workloads.gaussian(n, L, d, sigma=sigma)
    eps = 1e-13 if kernel == "poisson2d" else 1e-14
    u3 = oracle.evaluate(oracle.make_plan(kernel, d, n, L, eps=eps, padding=3), rho)
    ns = oracle.evaluate.__globals__["grid_points"](n, d)
    X = np.broadcast_arrays(*workloads.mesh(ns, L, d))
    r = np.sqrt(sum(x * x for x in X))
    ex = {"coulomb3d": cf.coulomb3d_gaussian, "coulomb2d": cf.coulomb2d_gaussian,
          "poisson2d": cf.poisson2d_gaussian}[kernel](r, sigma)
    assert relmax(u3, ex) <= 1e-13


@pytest.mark.parametrize("kernel,d", [("coulomb3d", 3), ("poisson2d", 2), ("dipolar3d", 3),
                                      ("davey_stewartson2d", 2)])
def test_padding3_adjoint_dot_and_symmetry(kernel, d):
    rng = np.random.default_rng(19)
    n, L = 10, 3.0
    dip = ((0.6, 0.8, 0.0), (0.0, 0.6, 0.8)) if kernel == "dipolar3d" else None
    plan = oracle.make_plan(kernel, d, n, L, eps=1e-13, dipole=dip, padding=3)
    r, v = rng.standard_normal((2,) + (n,) * d)
    Ar, Atv = oracle.evaluate(plan, r), oracle.adjoint(plan, v)
    lhs, rhs = float(np.sum(Ar * v)), float(np.sum(r * Atv))
    assert abs(lhs - rhs) <= 1e-14 * np.sqrt(np.sum(Ar ** 2) * np.sum(v ** 2))
    assert relmax(Atv, oracle.evaluate(plan, v)) < 1e-13


def test_padding3_separable_dft_equals_full_dft_and_needs_even_n():
    rng = np.random.default_rng(23)
    for shape in ((4, 4, 4), (6, 6)):
        x = rng.standard_normal(shape)
        assert relmax(dft.forward(x, p=3), dft.full_dft(x, p=3)) < 1e-13
    with pytest.raises(ValueError):
        oracle.make_plan("coulomb3d", 3, 9, 2.0, padding=3)


@pytest.mark.parametrize("kernel,d,n,L", [("coulomb3d", 3, 16, 4.0), ("coulomb3d", 3, (8, 12, 16), (2.0, 3.0, 4.0)),
                                          ("poisson2d", 2, 24, 6.0)])
def test_energy_parseval_reading(kernel, d, n, L):
    """The energy's Fourier-side reading: with u = crop(IDFT(S rho^) / M) on the padded grid
    (S = G + A0 - c2 |xi|^2, the oracle's own steps), sum_x rho u = (1/M) sum_k S |rho^|^2, and
    over the kept half kx = 0..n of the real transform the planes kx = 0 and kx = n count once,
    the others twice (S is even in every axis).  Checked against the oracle's energy by the
    grid sum in space (numpy FFTs, not the oracle's transforms)."""
    kw = {"eps": 1e-13} if kernel == "poisson2d" else {}
    plan = oracle.make_plan(kernel, d, n, L, **kw)
    rng = np.random.default_rng(5)
    rho = rng.standard_normal(plan.ns)
    E = oracle.energy(plan, rho)
    pad = np.zeros(tuple(2 * m for m in plan.ns))
    pad[tuple(slice(0, m) for m in plan.ns)] = rho
    S = full_spectrum(plan) + plan.A0 - plan.c2 * laplacian_symbol(plan)
    nx = plan.ns[-1]
    R = np.fft.rfftn(pad)                               # kx = 0..nx kept (last axis)
    w = np.full(nx + 1, 2.0)
    w[0] = w[nx] = 1.0
    M = float(np.prod(pad.shape))
    E_f = 0.5 * plan.cell * float(np.sum(w * S[..., :nx + 1] * np.abs(R) ** 2)) / M
    scale = 0.5 * plan.cell * float(np.sum(np.abs(rho * oracle.evaluate(plan, rho))))
    assert abs(E_f - E) <= 1e-14 * scale, (E_f, E)
