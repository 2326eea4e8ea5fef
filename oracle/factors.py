"""One-dimensional factor integrals of the kernel coefficients (Section 2.2).

The tensor-product coefficient of eq. (tensor) is, per axis and per Gaussian,
    g(tau, xi) = int_{-c}^{c} exp(-tau^2 y^2) cos(xi y) dy,   c = 2L,
taken at the padded-grid frequencies xi_k = pi k / (2L) = pi k / c (padding to
the box [-2L, 2L], the Remark after eq. (tensor)).  The paper evaluates these by
adaptive quadrature; the oracle writes the integral out as a composite
Gauss-Legendre rule on [0, c] with P = max(n, 8) equal panels of 20 nodes (at
most one half-period of cos(xi_k y) per panel for every k <= n), with two exact
special cases:
  * tau = 0:  g = 2c for k = 0 and exactly 0 otherwise (xi_k c = pi k);
  * tau c >= 6.5:  the box truncation is below 1e-19 relative, and g is the
    Gaussian Fourier transform sqrt(pi)/tau exp(-xi^2/(4 tau^2)).

At node y = c (p + s)/P of panel p the phase is xi_k y = pi k p / P + pi k s / P.
The first part is reduced exactly with integers ((k p) mod 2P), the second is
at most pi, and cos is formed by angle addition, so the phase error stays at
the level of one rounding even for k in the thousands.
"""

from __future__ import annotations

import math

import numpy as np

GL_NODES = 20
TAU_C_CLOSED = 6.5
_CHUNK = 32


def factor_1d(tau: np.ndarray, c: float, n: int) -> np.ndarray:
    """Matrix F[k, q] = g(tau_q, pi k / c) for k = 0..n (even in k)."""
    tau = np.asarray(tau, dtype=np.float64)
    k = np.arange(n + 1, dtype=np.float64)
    xi = math.pi * k / c
    F = np.zeros((n + 1, len(tau)))
    big = tau * c >= TAU_C_CLOSED
    zero = tau == 0.0
    mid = ~(big | zero)
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
