"""One-dimensional factor integrals of the kernel coefficients (Section 2.2).

The tensor-product coefficient of eq. (tensor) is, per axis and per Gaussian,
    g(tau, xi) = int_{-c}^{c} exp(-tau^2 y^2) cos(xi y) dy,   c = 2L,
taken at the padded-grid frequencies xi_k = 2 pi k / (p c), the frequencies of
the box [-p L, p L] the density is padded to: p = 2 (the Remark after eq.
(tensor): xi_k = pi k / c) or p = 3 (the box B_3 of eq. (FourSeriB3), the
integral still over B_2 as eq. (tensor) writes it: xi_k = 2 pi k / (3 c)).
The paper evaluates these by adaptive quadrature; the oracle writes the
integral out as a composite Gauss-Legendre rule on [0, c] with P equal panels
of 20 nodes, P = max(2 n / p, 8) for k = 0..n (at most one half-period of
cos(xi_k y) per panel), with three special cases:
  * tau = 0:  g = 2c for k = 0, 2 sin(xi_k c) / xi_k otherwise (exactly 0 for
    p = 2, where xi_k c = pi k);
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
summed in mpmath at 50 digits (the terms alternate and grow for small k).  For
p = 3 (a = 2 pi k / 3, sin a != 0) the same antiderivative is taken whole:
    m_m(a) = 2 Re[ e^{ia} sum_{j=0}^{m} (-1)^j m! / (m - j)! / (ia)^(j+1) - m! / (ia)^(m+1) ].

At node y = c (i + s)/P of panel i the phase is xi_k y = 2 pi k i / (p P) +
2 pi k s / (p P).  The first part is reduced exactly with integers
((2 k i) mod 2 p P), the second is at most pi, and cos is formed by angle
addition, so the phase error stays at the level of one rounding even for k in
the thousands.
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


@lru_cache(maxsize=8)
def _moments_general(n: int, p: int) -> np.ndarray:
    """m_2i(2 pi k / p) for k = 0..n, i = 0..SERIES_TERMS-1, from the whole antiderivative."""
    out = np.empty((n + 1, SERIES_TERMS))
    with mp.workdps(50):
        for k in range(n + 1):
            a = 2 * mp.pi * k / p
            for i in range(SERIES_TERMS):
                m = 2 * i
                if k == 0:
                    out[k, i] = 2.0 / (m + 1)
                    continue
                ia = mp.mpc(0, a)
                acc = mp.mpc(0)
                for j in range(m + 1):
                    acc += (-1) ** j * mp.factorial(m) / mp.factorial(m - j) / ia ** (j + 1)
                val = mp.exp(ia) * acc - mp.factorial(m) / ia ** (m + 1)
                out[k, i] = float(2 * mp.re(val))
    return out


def _factor_series(ts: np.ndarray, c: float, n: int, p: int = 2) -> np.ndarray:
    m = _moments(n) if p == 2 else _moments_general(n, p)    # (n+1, terms)
    x = (ts * c) ** 2                                        # (q,)
    coef = np.array([[(-xq) ** i / math.factorial(i) for xq in x] for i in range(SERIES_TERMS)])   # (terms, q)
    return c * (m @ coef)


def factor_1d(tau: np.ndarray, c: float, n: int, p: int = 2) -> np.ndarray:
    """Matrix F[k, q] = g(tau_q, 2 pi k / (p c)) for k = 0..n (even in k): the factors of
    the density padded to the box [-p c / 2, p c / 2], p = 2 or 3."""
    if p not in (2, 3):
        raise ValueError("padding factor p must be 2 or 3")
    tau = np.asarray(tau, dtype=np.float64)
    k = np.arange(n + 1, dtype=np.float64)
    xi = 2.0 * math.pi * k / (p * c)
    F = np.zeros((n + 1, len(tau)))
    big = tau * c >= TAU_C_CLOSED
    zero = tau == 0.0
    small = ~zero & (tau * c <= TAU_C_SERIES)
    mid = ~(big | zero | small)
    if np.any(small):
        F[:, small] = _factor_series(tau[small], c, n, p)
    if np.any(big):
        tb = tau[big]
        F[:, big] = math.sqrt(math.pi) / tb[None, :] * np.exp(-(xi[:, None] ** 2) / (4.0 * tb[None, :] ** 2))
    if np.any(zero):
        # 2 sin(xi_k c) / xi_k with xi_k c = 2 pi k / p, reduced exactly: pi ((2k) mod 2p) / p
        r = (2 * np.arange(1, n + 1)) % (2 * p)
        sn = np.where(r % p == 0, 0.0, np.sin(math.pi * r / p))
        col = np.concatenate([[2.0 * c], 2.0 * sn / xi[1:]])
        F[:, zero] = col[:, None]
    if np.any(mid):
        F[:, mid] = _factor_gl(tau[mid], c, n, p)
    return F


def _factor_gl(tm: np.ndarray, c: float, n: int, p: int = 2) -> np.ndarray:
    P = max((2 * n) // p, 8)
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
        m = (2 * kc[:, None] * p_idx[None, :]) % (2 * p * P)      # exact integer reduction
        A = math.pi * m.astype(np.float64) / (p * P)               # (k, P)
        B = math.pi * ((2 * kc[:, None]).astype(np.float64) * s[None, :]) / (p * P)   # (k, nodes), <= pi
        cA, sA, cB, sB = np.cos(A), np.sin(A), np.cos(B), np.sin(B)
        # sum_{p,i} gw[p,i,q] (cos A_kp cos B_ki - sin A_kp sin B_ki)
        Tc = np.einsum("ki,piq->kpq", cB, gw, optimize=True)
        Ts = np.einsum("ki,piq->kpq", sB, gw, optimize=True)
        # per-panel contributions, then a pairwise sum over the panels (last axis)
        contrib = cA[:, :, None] * Tc - sA[:, :, None] * Ts          # (k, P, q)
        out[k0:k0 + _CHUNK] = np.ascontiguousarray(contrib.transpose(0, 2, 1)).sum(axis=-1)
    return out
