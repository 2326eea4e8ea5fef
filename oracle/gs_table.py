"""Gaussian-sum tables by sinc quadrature (paper Section 3).

Coulomb kernel 1/r (Section 3.2, eqs. (Gauss_int), (GauInte), (sinc_quad)): start from the Gaussian
integral 1/r = (2/sqrt(pi)) int_0^inf exp(-r^2 tau^2) dtau, substitute
tau = sinh(t) (even integrand on the real line) and apply the sinc (infinite
trapezoidal) rule with step theta = c0 ln(S)/S, c0 = 2.1 (Remark after Prop. 1),
truncated to |k| <= S.  Folding k and -k gives S+1 terms:
    w_0 = theta/sqrt(pi),                tau_0 = 0,
    w_k = 2 theta cosh(k theta)/sqrt(pi), tau_k = sinh(k theta),  k = 1..S.

Poisson kernel ln r (Section 3.3).  The printed derivation is garbled; the
reading used here is Frullani's integral
    ln x = 1/2 int_0^inf (exp(-s) - exp(-s x^2)) ds / s,      x >= 1,
with the substitution s = ln(1 + exp(sinh t)) named in the paper (double
exponential decay on the real line) and the sinc rule with c0 = 1 over
k = -S..S (2S+1 nodes), giving
    ln x ~= C0 - sum_k wh_k exp(-s_k x^2),  wh_k = a_k/(2 s_k),
    a_k = theta cosh(t_k)/(1 + exp(-sinh t_k)),  C0 = sum_k wh_k exp(-s_k),
on x in [1, X], X = R/delta.  Nodes whose whole contribution on [1, X]
(about a_k X^2 / 2) is below 1e-3 eps are dropped: that is the stable evaluation
the paper asks for (otherwise s_k underflows and wh_k becomes 0/0).

Inverse powers 1/r^beta, 0 < beta < d (the Remark after eq. (GauInte)): the same
Gaussian integral with alpha = beta - 1,
    r^-beta = (2/Gamma(beta/2)) int_0^inf tau^(beta-1) exp(-r^2 tau^2) dtau
(eq. (Gauss_int) as printed lacks the factor 1/2 of int_0^inf; with alpha = 0 it
must give eq. (GauInte), which fixes it).  For beta != 1 the integrand is not even
in tau, so the sinh substitution does not apply; the reading taken is the double-
exponential substitution tau = exp(t - e^-t) (decay exp(-beta e^-t) as t -> -inf,
exp(-r^2 e^2t) as t -> inf), sinc rule with step theta = c0 ln(S)/S, c0 = 2, over
k = -S..S:
    w_k = (2/Gamma(beta/2)) theta tau_k^beta (1 + e^-t_k),   tau_k = exp(t_k - e^-t_k),
keeping the nodes whose largest contribution r^beta w_k exp(-tau_k^2 r^2) on the
fit interval exceeds 1e-3 eps.

S is the smallest value whose maximum error on 100001 log-spaced points of the
fit interval is <= eps: relative error of 1/r on [delta, R] (the paper's E_rel),
absolute error of ln on [delta, R] (E_abs), both in box-rescaled units
(Section 2.1, lengths in units of the largest half-width L).  R is the largest
distance |y| between two points of the box: 2 sqrt(d) for the cube (the paper
writes [delta, 2]; |y| over [-2,2]^d reaches 2 sqrt(d), so the interval is
widened to it) and 2 sqrt(sum_j (L_j/L)^2) for a rectangular box (Section 2.5,
where the short axis is eta times the others).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

NPTS = 100001          # check points on the fit interval
SUBSET = 50            # every 50th point: a cheap necessary test
S_MAX = 4000


def _theta(S: int, c0: float) -> float:
    return c0 * math.log(S) / S


def coulomb_nodes(S: int, c0: float = 2.1):
    """Rescaled 1/r table (w~, tau~) with S+1 terms, q = 0 the tau = 0 term."""
    th = _theta(S, c0)
    k = np.arange(S + 1, dtype=np.float64)
    w = 2.0 * th * np.cosh(k * th) / math.sqrt(math.pi)
    w[0] = th / math.sqrt(math.pi)
    tau = np.sinh(k * th)
    tau[0] = 0.0
    return w, tau


def _sum_gauss(w, tau2, r2):
    """sum_q w_q exp(-tau2_q r2), summed from the largest tau down."""
    acc = np.zeros_like(r2)
    for q in range(len(w) - 1, -1, -1):
        acc += w[q] * np.exp(-tau2[q] * r2)
    return acc


def coulomb_error(S: int, lo: float, hi: float, c0: float = 2.1, pts=None) -> float:
    w, tau = coulomb_nodes(S, c0)
    r = np.geomspace(lo, hi, NPTS) if pts is None else pts
    return float(np.max(np.abs(1.0 - r * _sum_gauss(w, tau * tau, r * r))))


def _smallest_S(err_fn, pts_full) -> int:
    sub = pts_full[::SUBSET]
    for S in range(2, S_MAX + 1):
        if err_fn(S, sub) > _EPS_BOX[0]:
            continue
        if err_fn(S, pts_full) <= _EPS_BOX[0]:
            return S
    raise ValueError("requested accuracy not reachable by the sinc table")


_EPS_BOX = [0.0]


def coulomb_table(d: int, delta_rel: float, eps: float, c0: float = 2.1, hi: float | None = None):
    """Smallest-S 1/r table meeting E_rel <= eps on [delta_rel, hi] (default 2 sqrt(d))."""
    hi = 2.0 * math.sqrt(d) if hi is None else hi
    pts = np.geomspace(delta_rel, hi, NPTS)
    _EPS_BOX[0] = eps
    S = _smallest_S(lambda S, p: coulomb_error(S, 0, 0, c0, pts=p), pts)
    w, tau = coulomb_nodes(S, c0)
    return w, tau, S


def power_nodes(beta: float, S: int, lo: float, hi: float, eps: float, c0: float = 2.0):
    """Rescaled 1/r^beta table (w~, tau~) on [lo, hi] with the negligible nodes dropped."""
    th = _theta(S, c0)
    t = np.arange(-S, S + 1, dtype=np.float64) * th
    tau = np.exp(t - np.exp(-t))
    w = (2.0 / math.gamma(beta / 2.0)) * th * tau ** beta * (1.0 + np.exp(-t))
    with np.errstate(divide="ignore", over="ignore"):
        rstar = np.clip(math.sqrt(beta / 2.0) / tau, lo, hi)   # where r^beta e^(-tau^2 r^2) peaks
    keep = w * rstar ** beta * np.exp(-(tau * rstar) ** 2) > 1e-3 * eps
    return w[keep], tau[keep]


def power_error(beta: float, S: int, lo: float, hi: float, eps: float, c0: float = 2.0, pts=None) -> float:
    w, tau = power_nodes(beta, S, lo, hi, eps, c0)
    r = np.geomspace(lo, hi, NPTS) if pts is None else pts
    return float(np.max(np.abs(1.0 - r ** beta * _sum_gauss(w[np.argsort(tau)], np.sort(tau) ** 2, r * r))))


def power_table(beta: float, delta_rel: float, eps: float, hi: float, c0: float = 2.0):
    """Smallest-S 1/r^beta table meeting the relative error eps on [delta_rel, hi]."""
    pts = np.geomspace(delta_rel, hi, NPTS)
    _EPS_BOX[0] = eps
    S = _smallest_S(lambda S, p: power_error(beta, S, delta_rel, hi, eps, c0, pts=p), pts)
    w, tau = power_nodes(beta, S, delta_rel, hi, eps, c0)
    return w, tau, S


def poisson_nodes(S: int, X: float, eps: float, c0: float = 1.0):
    """Rescaled ln table: returns (C0, wh, s) with the negligible nodes dropped."""
    th = _theta(S, c0)
    t = np.arange(-S, S + 1, dtype=np.float64) * th
    sh = np.sinh(t)
    # s = ln(1 + e^sh) without overflow or cancellation
    s = np.where(sh > 0, sh + np.log1p(np.exp(-np.abs(sh))), np.log1p(np.exp(np.minimum(sh, 0.0))))
    # 1/(1 + e^-sh) evaluated stably on both sides
    sig = np.where(sh >= 0, 1.0 / (1.0 + np.exp(-np.abs(sh))),
                   np.exp(-np.abs(sh)) / (1.0 + np.exp(-np.abs(sh))))
    a = th * np.cosh(t) * sig
    keep = a * X * X / 2.0 > 1e-3 * eps
    s, a = s[keep], a[keep]
    wh = a / (2.0 * s)
    C0 = float(np.sum(wh * np.exp(-s)))
    return C0, wh, s


def poisson_error(S: int, X: float, eps: float, c0: float = 1.0, pts=None) -> float:
    """max |ln x - (C0 - sum wh exp(-s x^2))| with the approximation summed as
    sum_k wh_k (exp(-s_k) - exp(-s_k x^2)): positive terms, no cancellation
    against the constant, so the measured error is the quadrature error."""
    C0, wh, s = poisson_nodes(S, X, eps, c0)
    x2m1 = pts * pts - 1.0
    acc = np.zeros_like(pts)
    for q in range(len(wh) - 1, -1, -1):
        acc += wh[q] * (-np.exp(-s[q]) * np.expm1(-s[q] * x2m1))
    return float(np.max(np.abs(np.log(pts) - acc)))


def poisson_table(delta_rel: float, eps: float, c0: float = 1.0, hi: float | None = None):
    """Smallest-S ln table meeting E_abs <= eps for r in [delta_rel, hi] (default
    2 sqrt(2)), i.e. x = r/delta_rel in [1, hi/delta_rel]."""
    hi = 2.0 * math.sqrt(2.0) if hi is None else hi
    X = hi / delta_rel
    pts = np.geomspace(1.0, X, NPTS)
    _EPS_BOX[0] = eps
    S = _smallest_S(lambda S, p: poisson_error(S, X, eps, c0, pts=p), pts)
    C0, wh, s = poisson_nodes(S, X, eps, c0)
    return C0, wh, s, S


@dataclass
class GSTable:
    """Physical-unit table U_GS(r) = sum_q w[q] exp(-tau[q]^2 r^2), q = 0 has tau = 0."""

    w: np.ndarray
    tau: np.ndarray
    S: int
    delta: float         # physical near-field radius delta_rel * L
    kernel: str
    d: int
    L: float             # length unit: the largest half-width of the box


def box_half_widths(L, d: int) -> tuple:
    """Per-axis half-widths (C order: z, y, x in 3D; y, x in 2D) from a scalar or a sequence."""
    if np.ndim(L) == 0:
        return (float(L),) * d
    Ls = tuple(float(v) for v in L)
    if len(Ls) != d:
        raise ValueError("one half-width per axis")
    return Ls


def fit_interval_end(Ls) -> float:
    """R = largest |y| over the difference box, in units of the largest half-width."""
    Lu = max(Ls)
    return 2.0 * math.sqrt(sum((v / Lu) ** 2 for v in Ls))


def physical_table(kernel: str, d: int, L, eps: float, delta_rel: float = 1e-4, beta: float | None = None) -> GSTable:
    """Table for U in physical units on the box prod_j [-L_j, L_j] (Section 2.1
    rescaling, with the largest half-width L as the length unit; Section 2.5 for
    rectangular boxes).

    Coulomb: 1/r = (1/L)(1/r~) with r~ = r/L, so w = kappa w~/L, tau = tau~/L,
    kappa = 1/(4 pi) (3D) or 1/(2 pi) (2D).  Poisson: -ln(r)/(2 pi) with
    r = delta x, delta = delta_rel L: w_0 = -(ln delta + C0)/(2 pi), tau_0 = 0,
    w_k = wh_k/(2 pi), tau_k = sqrt(s_k)/delta.  Inverse power r^-beta = L^-beta r~^-beta:
    w = w~/L^beta, tau = tau~/L.  The near-field ball must fit the
    shortest axis (Section 2.5: delta below eta): delta_rel < min_j L_j / L.
    """
    dd = 3 if kernel in ("coulomb3d", "dipolar3d") else (
        2 if kernel in ("coulomb2d", "poisson2d", "davey_stewartson2d") else d)
    Ls = box_half_widths(L, dd)
    L = max(Ls)
    if not delta_rel < min(Ls) / L:
        raise ValueError("delta_rel must be below the shortest half-width over the largest")
    hi = fit_interval_end(Ls)
    delta = delta_rel * L
    if kernel in ("coulomb3d", "coulomb2d", "dipolar3d"):
        kappa = 1.0 / (4.0 * math.pi) if dd == 3 else 1.0 / (2.0 * math.pi)
        wt, tt, S = coulomb_table(dd, delta_rel, eps, hi=hi)
        return GSTable(kappa * wt / L, tt / L, S, delta, kernel, dd, L)
    if kernel == "inverse_power":
        if beta is None or not 0.0 < beta < dd:
            raise ValueError("inverse_power needs 0 < beta < d")
        wt, tt, S = power_table(beta, delta_rel, eps, hi)
        return GSTable(wt / L ** beta, tt / L, S, delta, kernel, dd, L)
    if kernel in ("poisson2d", "davey_stewartson2d"):
        # the Davey-Stewartson potential convolves the same logarithmic kernel
        C0, wh, s, S = poisson_table(delta_rel, eps, hi=hi)
        w = np.concatenate([[-(math.log(delta) + C0) / (2.0 * math.pi)], wh / (2.0 * math.pi)])
        tau = np.concatenate([[0.0], np.sqrt(s) / delta])
        return GSTable(w, tau, S, delta, kernel, 2, L)
    raise ValueError(kernel)


def custom_table(w, tau, d: int, L, kernel: str = "gaussian_sum") -> GSTable:
    """A user-given Gaussian sum (test hook): no Taylor correction is applied."""
    return GSTable(np.asarray(w, float), np.asarray(tau, float), len(w) - 1, 0.0, kernel, d,
                   max(box_half_widths(L, d)))
