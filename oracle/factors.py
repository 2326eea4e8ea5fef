"""One-dimensional factor integrals of the kernel coefficients (Section 2.2).

The tensor-product coefficient of eq. (tensor) is, per axis and per Gaussian,
    g(tau, xi) = int_{-c}^{c} exp(-tau^2 y^2) cos(xi y) dy,   c = 2L,
taken at the padded-grid frequencies xi_k = pi k / (2L) = pi k / c (padding to
the box [-2L, 2L], the Remark after eq. (tensor)).  The paper evaluates these by
adaptive quadrature; the oracle writes the integral out as a composite
Gauss-Legendre rule on [0, c] with P = max(n, 8) equal panels of 20 nodes (at
most one half-period of cos(xi_k y) per panel for every k <= n), with three
special cases:
  * tau = 0:  g = 2c for k = 0 and exactly 0 otherwise (xi_k c = pi k);
  * tau c >= 6.5:  the box truncation is below 1e-19 relative, and g is the
    Gaussian Fourier transform sqrt(pi)/tau exp(-xi^2/(4 tau^2));
  * tau c <= 0.05:  the power series of the Gaussian in tau^2 integrated term by
    term, g = c sum_i (-(tau c)^2)^i / i! m_2i(pi k) with the exact moments
    m_2i(a) = int_{-1}^{1} t^2i cos(a t) dt.  There the value at k >= 1 is of the
    size (tau c)^2 c, far below the rounding noise (about 1e-16 c) that a
    quadrature of the oscillating integrand leaves; the series has none.
The moments come from the antiderivative of t^m e^{iat} (m even, a = pi k >= 1,
e^{ia} = e^{-ia} = (-1)^k):
    m_m(pi k) = (-1)^k sum_{l=1}^{m/2} 2 (-1)^(l+1) m! / (m - 2l + 1)! / (pi k)^(2l),
    m_m(0) = 2 / (m + 1),
summed in mpmath at 50 digits (the terms alternate and grow for small k).

At node y = c (p + s)/P of panel p the phase is xi_k y = pi k p / P + pi k s / P.
The first part is reduced exactly with integers ((k p) mod 2P), the second is
at most pi, and cos is formed by angle addition, so the phase error stays at
the level of one rounding even for k in the thousands.
"""

from __future__ import annotations

import math
from functools import lru_cache

import mpmath as mp
import numpy as np

GL_NODES = 20
TAU_C_CLOSED = 6.5
TAU_C_SERIES = 0.05
SERIES_TERMS = 12          # (0.05^2)^12 / 12! < 1e-40
_CHUNK = 32


@lru_cache(maxsize=8)
def _moments(n: int) -> np.ndarray:
    """m_2i(pi k) for k = 0..n, i = 0..SERIES_TERMS-1, as float64 (n+1, SERIES_TERMS)."""
    out = np.empty((n + 1, SERIES_TERMS))
    with mp.workdps(50):
        for k in range(n + 1):
            for i in range(SERIES_TERMS):
                m = 2 * i
                if k == 0:
                    out[k, i] = 2.0 / (m + 1)
                    continue
                a = mp.pi * k
                acc = mp.mpf(0)
                for l in range(1, m // 2 + 1):
                    acc += 2 * (-1) ** (l + 1) * mp.factorial(m) / mp.factorial(m - 2 * l + 1) / a ** (2 * l)
                out[k, i] = float((-1) ** k * acc)
    return out


def _factor_series(ts: np.ndarray, c: float, n: int) -> np.ndarray:
    m = _moments(n)                                          # (n+1, terms)
    x = (ts * c) ** 2                                        # (q,)
    coef = np.array([[(-xq) ** i / math.factorial(i) for xq in x] for i in range(SERIES_TERMS)])   # (terms, q)
    return c * (m @ coef)


def factor_1d(tau: np.ndarray, c: float, n: int) -> np.ndarray:
    """Matrix F[k, q] = g(tau_q, pi k / c) for k = 0..n (even in k)."""
    tau = np.asarray(tau, dtype=np.float64)
    k = np.arange(n + 1, dtype=np.float64)
    xi = math.pi * k / c
    F = np.zeros((n + 1, len(tau)))
    big = tau * c >= TAU_C_CLOSED
    zero = tau == 0.0
    small = ~zero & (tau * c <= TAU_C_SERIES)
    mid = ~(big | zero | small)
    if np.any(small):
        F[:, small] = _factor_series(tau[small], c, n)
    if np.any(big):
        tb = tau[big]
        F[:, big] = math.sqrt(math.pi) / tb[None, :] * np.exp(-(xi[:, None] ** 2) / (4.0 * tb[None, :] ** 2))
    if np.any(zero):
        F[0, zero] = 2.0 * c
    if np.any(mid):
        F[:, mid] = _factor_gl(tau[mid], c, n)
    return F


def _factor_gl(tm: np.ndarray, c: float, n: int) -> np.ndarray:
    P = max(n, 8)
    xg, wg = np.polynomial.legendre.leggauss(GL_NODES)
    s = 0.5 * (xg + 1.0)                                   # node offsets in a panel, (0, 1)
    hp = c / P
    y = hp * (np.arange(P)[:, None] + s[None, :])          # (P, nodes)
    # 2 * (GL weight) * Gaussian, per panel, node, Gaussian:  (P, nodes, q)
    gw = (2.0 * 0.5 * hp * wg)[None, :, None] * np.exp(-(tm[None, None, :] ** 2) * (y[:, :, None] ** 2))
    kk = np.arange(n + 1, dtype=np.int64)
    out = np.empty((n + 1, len(tm)))
    p_idx = np.arange(P, dtype=np.int64)
    for k0 in range(0, n + 1, _CHUNK):
        kc = kk[k0:k0 + _CHUNK]
        m = (kc[:, None] * p_idx[None, :]) % (2 * P)       # exact integer reduction
        A = math.pi * m.astype(np.float64) / P             # (k, P)
        B = math.pi * (kc[:, None].astype(np.float64) * s[None, :]) / P   # (k, nodes), <= pi
        cA, sA, cB, sB = np.cos(A), np.sin(A), np.cos(B), np.sin(B)
        # sum_{p,i} gw[p,i,q] (cos A_kp cos B_ki - sin A_kp sin B_ki)
        Tc = np.einsum("ki,piq->kpq", cB, gw, optimize=True)
        Ts = np.einsum("ki,piq->kpq", sB, gw, optimize=True)
        # per-panel contributions, then a pairwise sum over the panels (last axis)
        contrib = cA[:, :, None] * Tc - sA[:, :, None] * Ts          # (k, P, q)
        out[k0:k0 + _CHUNK] = np.ascontiguousarray(contrib.transpose(0, 2, 1)).sum(axis=-1)
    return out
