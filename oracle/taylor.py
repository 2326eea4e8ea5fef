"""Near-field Taylor correction constants (Section 2.3, eq. (taylor)).

In the ball |y| < delta the density rho(x - y) is replaced by its third-order
Taylor polynomial.  Integrating against the radial weight (U - U_GS)(|y|), the
odd terms and the off-diagonal Hessian terms vanish, and each diagonal term
contributes (1/d) |y|^2 of the radial moment, so
    I21~(x) = A0 rho(x) + c2 (Laplacian rho)(x),
    A0 = |S^{d-1}| int_0^delta r^{d-1} (U - U_GS)(r) dr,
    c2 = |S^{d-1}| / (2d) int_0^delta r^{d+1} (U - U_GS)(r) dr,
with |S^{d-1}| = 2 pi^{d/2} / Gamma(d/2).  The paper never prints these
constants; the expressions above follow from its derivation.

The U parts are elementary (kernel constants included):
    3D Coulomb 1/(4 pi r):      int r^2 U = delta^2/(8 pi),   int r^4 U = delta^4/(16 pi)
    2D Coulomb 1/(2 pi r):      int r U   = delta/(2 pi),     int r^3 U = delta^3/(6 pi)
    inverse power r^-beta:      int r^m U = delta^(m+1-beta)/(m+1-beta)    (m = d-1, d+1)
    2D Poisson -ln r/(2 pi):    int r U   = (delta^2/4 - delta^2 ln(delta)/2)/(2 pi),
                                int r^3 U = (delta^4/16 - delta^4 ln(delta)/4)/(2 pi)
and the Gaussian parts are lower incomplete gamma functions,
    gamma_m(tau) = int_0^delta r^m exp(-tau^2 r^2) dr
                 = gammainc((m+1)/2, 0, tau^2 delta^2) / (2 tau^(m+1)),
    gamma_m(0)   = delta^(m+1)/(m+1),
evaluated with mpmath at 40 digits.
"""

from __future__ import annotations

import math

import mpmath as mp


def sphere_area(d: int) -> float:
    return float(2 * mp.pi ** (mp.mpf(d) / 2) / mp.gamma(mp.mpf(d) / 2))


def _u_moment(kernel: str, m: int, delta, beta=None):
    """int_0^delta r^m U(r) dr (mpmath)."""
    dl = mp.mpf(delta)
    if kernel == "inverse_power":                        # int_0^delta r^(m - beta) dr
        e = m + 1 - mp.mpf(beta)
        return dl ** e / e
    if kernel in ("coulomb3d", "dipolar3d"):
        return dl ** m / (4 * mp.pi * m)                 # int r^{m-1}/(4 pi) dr
    if kernel == "coulomb2d":
        return dl ** m / (2 * mp.pi * m)
    if kernel in ("poisson2d", "davey_stewartson2d"):
        # -(1/2pi) int_0^delta r^m ln r dr = -(1/2pi) [delta^{m+1}(ln delta/(m+1) - 1/(m+1)^2)]
        a = m + 1
        return -(dl ** a) * (mp.log(dl) / a - mp.mpf(1) / a ** 2) / (2 * mp.pi)
    raise ValueError(kernel)


def gamma_moment(m: int, tau, delta):
    t = mp.mpf(tau)
    dl = mp.mpf(delta)
    if t == 0:
        return dl ** (m + 1) / (m + 1)
    a = mp.mpf(m + 1) / 2
    return mp.gammainc(a, 0, (t * dl) ** 2) / (2 * t ** (m + 1))


def taylor_constants(kernel: str, d: int, delta: float, w, tau, beta=None):
    """(A0, c2) for the table (w, tau) and the physical radius delta (beta: the exponent
    of the inverse-power kernel r^-beta, whose moments need beta < d)."""
    with mp.workdps(40):
        area = 2 * mp.pi ** (mp.mpf(d) / 2) / mp.gamma(mp.mpf(d) / 2)
        m0, m2 = d - 1, d + 1
        s0 = _u_moment(kernel, m0, delta, beta)
        s2 = _u_moment(kernel, m2, delta, beta)
        for wq, tq in zip(w, tau):
            s0 -= mp.mpf(float(wq)) * gamma_moment(m0, float(tq), delta)
            s2 -= mp.mpf(float(wq)) * gamma_moment(m2, float(tq), delta)
        A0 = area * s0
        c2 = area * s2 / (2 * d)
        return float(A0), float(c2)
