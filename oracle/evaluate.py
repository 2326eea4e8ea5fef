"""The evaluation itself, step by step as in Algorithm 1 (Section 2.4).

Precomputation (plan):
  1. Gaussian-sum table of the kernel (Section 3; `gs_table`).
  2. The stored coefficient sums  G_k = sum_q w_q prod_j g_q(xi_{k_j})  of
     eqs. (I1FFT), (tensor), from the one-dimensional factors (`factors`).  G is even
     in every index, so it is formed on the octant k_j in [0, n] and extended.
  3. The Taylor constants A0, c2 of Section 2.3 (`taylor`).
Actual computation (evaluate):
  1. rho~ = DFT(pad(rho))                                (eqs. (FourSeriB3), (rho_hat))
  2. I1   = (1/M) crop(IDFT(G . rho~))                   (eq. (I1FFT))
  3. Lap  = (1/M) crop(IDFT(-|xi|^2 . rho~))             (spectral Laplacian; or, with
     laplacian="unpadded", the spectral Laplacian on the density's own grid,
     period 2 L_j: DFT_n, -|xi'|^2 with xi'_k = pi k / L_j, k in [-n_j/2, n_j/2), IDFT_n / prod n_j)
  4. I21~ = A0 rho + c2 Lap                              (eq. (taylor))
  5. u    = I1 + I21~
with M = prod_j 2 n_j.  The Laplacian is taken on the padded grid with the Nyquist
mode kept (|xi| = pi/h there).

Padding (padding=3): the body of Section 2.2 pads the density to B_3 = [-3L, 3L]
(eq. (FourSeriB3), n~ = 3n): every 2 above becomes 3, i.e. transforms of length
3 n_j with n_j non-zero inputs, xi_k = pi k / (3 L_j) for k in [-3n_j/2, 3n_j/2),
M = prod_j 3 n_j, while the factor integrals stay over [-2 L_j, 2 L_j] as eq.
(tensor) writes them (at the new frequencies).  n_j must be even (the index range
of eq. (FourSeriB3)).  The default, padding=2, is the Remark after eq. (tensor).

Rectangular boxes (Section 2.5): the box is prod_j [-L_j, L_j] with n_j points on
axis j (one n for every axis, or one per axis), so h_j = 2 L_j / n_j, the padded
grid has 2 n_j points and xi^(j)_k = pi k / (2 L_j); the factors of
eq. (tensor_ani) are the one-dimensional integrals over [-2 L_j, 2 L_j] at those
frequencies (k = 0..n_j), the Laplacian symbol is sum_j (xi^(j))^2,
M = prod_j 2 n_j, and the Gaussian-sum table is fitted on the rescaled distances
of that box (`gs_table`).  The
printed phase factor of eq. (tensor_ani)'s companion formula carries a stray
epsilon where the axis ratio eta is meant; with eta the short axis is simply an
axis of half-width eta L, which is what per-axis half-widths express.

Dipolar potential (Section 2.4): u = -(n.m) rho - 3 Coul3D(d_n d_m rho), the
source d_n d_m rho having padded coefficients -(n.xi)(m.xi) rho~.  Davey-Stewartson
potential (the remark closing Section 2.4 and Example 4.5): u = Poisson2D(d_xx rho),
the source having padded coefficients -xi_x^2 rho~ (an even symbol: the Nyquist
frequency keeps pi/h_x).  In the cross
terms xi_i xi_j (i != j) the Nyquist frequency is taken as 0 (an odd symbol has
no value there that keeps the result real); squares keep (pi/h)^2.

The operator is real, linear and, the kernel being even, symmetric.  `adjoint`
applies the transposed steps literally (pad and crop exchanged, DFT signs
flipped), `energy` is 1/2 h^d sum rho u, and its rho-gradient is h^d u.
`energy_gradient_params` carries that gradient to the parameters of a Gaussian
mixture density by the chain rule.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import dft
from .factors import factor_1d
from .gs_table import GSTable, box_half_widths, custom_table, physical_table
from .taylor import taylor_constants

COULOMB_LIKE = ("coulomb3d", "coulomb2d", "poisson2d", "dipolar3d", "davey_stewartson2d", "inverse_power")


@dataclass
class OraclePlan:
    kernel: str
    d: int
    n: int                  # points per axis (the largest, when the axes differ)
    L: float                # largest half-width (the table's length unit)
    table: GSTable
    F: np.ndarray           # (n+1, Q) one-dimensional factors of the last axis (x)
    G_oct: np.ndarray       # (n+1)^d regular-part coefficients, array axis order
    A0: float
    c2: float
    dipole_n: tuple | None = None
    dipole_m: tuple | None = None
    Ls: tuple = ()          # per-axis half-widths, C order (z, y, x / y, x)
    Fs: tuple = ()          # per-axis factor matrices, C order
    beta: float | None = None   # exponent of the inverse-power kernel r^-beta
    ns: tuple = ()          # points per axis, C order
    laplacian: str = "padded"   # grid of the Taylor term's Laplacian: "padded" or "unpadded"
    padding: int = 2        # the density is zero-padded to [-p L, p L], p = 2 or 3

    @property
    def h(self) -> float:
        """Grid step of a cubic box (use `hs` for rectangular ones)."""
        if len(set(self.hs)) > 1:
            raise ValueError("rectangular box: the grid step differs per axis")
        return self.hs[0]

    @property
    def hs(self) -> tuple:
        return tuple(2.0 * v / m for v, m in zip(self.Ls, self.ns))

    @property
    def cell(self) -> float:
        """Volume of a grid cell, prod_j h_j."""
        return float(np.prod(self.hs))

    @property
    def M(self) -> int:
        return int(np.prod([self.padding * m for m in self.ns]))


def make_plan(kernel: str, d: int, n, L, eps: float = 1e-14,
              delta_rel: float = 1e-4, custom=None, dipole=None, beta: float | None = None,
              laplacian: str = "padded", padding: int = 2) -> OraclePlan:
    """n, L: one value for every axis (the cube [-L, L]^d with n^d points), or one per axis
    in C order; beta: the exponent of kernel "inverse_power" (U = |x|^-beta, 0 < beta < d);
    laplacian: the grid on which the Taylor term takes the density's Laplacian (Algorithm 1
    step 3): "padded" (the 2n grid of the convolution) or "unpadded" (the density's own
    grid, periodic); padding: 2 (the box [-2L, 2L]) or 3 (B_3, every n even)."""
    if laplacian not in ("padded", "unpadded"):
        raise ValueError("laplacian: padded or unpadded")
    if padding not in (2, 3):
        raise ValueError("padding: 2 or 3")
    Ls = box_half_widths(L, d)
    ns = grid_points(n, d)
    if padding == 3 and any(m % 2 for m in ns):
        raise ValueError("padding 3 needs an even number of points per axis")
    p = padding
    if kernel == "gaussian_sum":
        w, tau = custom
        table = custom_table(w, tau, d, Ls)
    else:
        table = physical_table(kernel, d, Ls, eps, delta_rel, beta=beta)
        if table.d != d:
            raise ValueError("kernel and dimension disagree")
    # factors on the octant k = 0..p n / 2 of the padded frequencies
    Fs = tuple(factor_1d(table.tau, 2.0 * Lj, p * m // 2, p) for Lj, m in zip(Ls, ns))
    # G[i0][i1]([i2]) = sum_q w_q F_0[i0, q] F_1[i1, q] (F_2[i2, q]), array axes
    Fw = Fs[0] * table.w[None, :]
    if d == 2:
        G = Fw @ Fs[1].T
    else:
        G = np.empty(tuple(p * m // 2 + 1 for m in ns))
        for a in range(p * ns[0] // 2 + 1):
            G[a] = (Fw[a][None, :] * Fs[1]) @ Fs[2].T
    if kernel == "gaussian_sum":
        A0, c2 = 0.0, 0.0
    else:
        A0, c2 = taylor_constants(kernel, d, table.delta, table.w, table.tau, beta)
    dn = dm = None
    if kernel == "dipolar3d":
        dn, dm = dipole
    return OraclePlan(kernel, d, max(ns), table.L, table, Fs[-1], G, A0, c2, dn, dm, Ls, Fs, beta, ns, laplacian,
                      padding)


def grid_points(n, d: int) -> tuple:
    """Points per axis (C order) from one value or a sequence."""
    if np.ndim(n) == 0:
        return (int(n),) * d
    ns = tuple(int(v) for v in n)
    if len(ns) != d:
        raise ValueError("one n per axis")
    return ns


def padded_frequencies(n: int, L: float, odd: bool = False, p: int = 2) -> np.ndarray:
    """xi_k = pi k'/(p L) for padded index k = 0..p n-1, k' = k - p n for k >= p n / 2.
    The Nyquist index k = p n / 2 carries -pi n/(2L) (even use) or 0 (odd use)."""
    N = p * n
    k = np.arange(N)
    ks = np.where(k < N // 2, k, k - N).astype(np.float64)
    xi = math.pi * ks / (p * L)
    if odd:
        xi[N // 2] = 0.0
    return xi


def _fold_index(n: int, p: int = 2) -> np.ndarray:
    k = np.arange(p * n)
    return np.minimum(k, p * n - k)


def full_spectrum(plan: OraclePlan) -> np.ndarray:
    return plan.G_oct[np.ix_(*[_fold_index(m, plan.padding) for m in plan.ns])]


def _axes_vectors(plan: OraclePlan, odd: bool):
    """Per-axis xi arrays shaped to broadcast over the [z][y][x] (or [y][x]) grid,
    returned in vector-component order (x, y[, z])."""
    d = plan.d
    out = []
    for comp in range(d):
        ax = d - 1 - comp                       # x is the last array axis
        xi = padded_frequencies(plan.ns[ax], plan.Ls[ax], odd, plan.padding)
        shape = [1] * d
        shape[ax] = plan.padding * plan.ns[ax]
        out.append(xi.reshape(shape))
    return out


def laplacian_symbol(plan: OraclePlan) -> np.ndarray:
    xs = _axes_vectors(plan, odd=False)
    return sum(x * x for x in xs)


def dipolar_symbol(plan: OraclePlan) -> np.ndarray:
    """(n.xi)(m.xi) with squares from the even xi and cross terms from the odd xi."""
    ev = _axes_vectors(plan, odd=False)
    od = _axes_vectors(plan, odd=True)
    nv, mv = plan.dipole_n, plan.dipole_m
    sym = 0.0
    for i in range(3):
        for j in range(3):
            if i == j:
                sym = sym + nv[i] * mv[i] * ev[i] * ev[i]
            else:
                sym = sym + nv[i] * mv[j] * od[i] * od[j]
    return sym


def periodic_laplacian(plan: OraclePlan, f: np.ndarray) -> np.ndarray:
    """Spectral Laplacian of f on its own grid (period 2 L_j on axis j): symbol
    -sum_j (pi k_j / L_j)^2 with k_j in [-n_j/2, n_j/2) (the Nyquist mode k = -n_j/2 kept)."""
    sym = 0.0
    for ax, (m, Lj) in enumerate(zip(plan.ns, plan.Ls)):
        k = np.arange(m)
        ks = np.where(k < m // 2, k, k - m).astype(np.float64)
        xi = math.pi * ks / Lj
        shape = [1] * plan.d
        shape[ax] = m
        sym = sym + (xi * xi).reshape(shape)
    return dft.periodic(-sym * dft.periodic(f), sign=+1).real / float(np.prod(plan.ns))


def _coulomb_steps(plan: OraclePlan, rt: np.ndarray, f: np.ndarray, sign: int = +1) -> np.ndarray:
    """I1 + A0 f + c2 Lap f for padded coefficients rt of the source f."""
    M, p = plan.M, plan.padding
    G = full_spectrum(plan)
    I1 = dft.inverse(G * rt, sign, p).real / M
    if plan.A0 == 0.0 and plan.c2 == 0.0:
        return I1
    if plan.laplacian == "unpadded":
        lap = periodic_laplacian(plan, f)
    else:
        lap = dft.inverse(-laplacian_symbol(plan) * rt, sign, p).real / M
    return I1 + plan.A0 * f + plan.c2 * lap


def ds_symbol(plan: OraclePlan) -> np.ndarray:
    """-xi_x^2 on the padded grid: the symbol of d_xx (x the last array axis)."""
    xs = _axes_vectors(plan, odd=False)
    return -(xs[0] * xs[0])


def evaluate(plan: OraclePlan, rho: np.ndarray) -> np.ndarray:
    rho = np.asarray(rho, dtype=np.float64)
    assert rho.shape == tuple(plan.ns)
    p = plan.padding
    rt = dft.forward(rho, p=p)
    if plan.kernel == "davey_stewartson2d":
        src_t = ds_symbol(plan) * rt
        src = dft.inverse(src_t, p=p).real / plan.M
        return _coulomb_steps(plan, src_t, src)
    if plan.kernel != "dipolar3d":
        return _coulomb_steps(plan, rt, rho)
    src_t = -dipolar_symbol(plan) * rt
    src = dft.inverse(src_t, p=p).real / plan.M
    nm = float(np.dot(plan.dipole_n, plan.dipole_m))
    return -nm * rho - 3.0 * _coulomb_steps(plan, src_t, src)


def adjoint(plan: OraclePlan, v: np.ndarray) -> np.ndarray:
    """Transpose of `evaluate` as a real linear map: every step transposed in
    reverse order (crop -> zero-pad, pad -> crop, DFT sign flipped)."""
    v = np.asarray(v, dtype=np.float64)
    p = plan.padding
    vt = dft.forward(v, sign=+1, p=p)                  # transpose of the crop-inverse
    M = plan.M
    unpadded = plan.laplacian == "unpadded"
    # the periodic Laplacian on the density's grid is symmetric: its transpose is itself
    lap_v = periodic_laplacian(plan, v) if unpadded else None
    lap_t = 0.0 if unpadded else -laplacian_symbol(plan) * vt
    if plan.kernel == "davey_stewartson2d":
        # transpose of rho -> [I1 + A0 f + c2 Lap f](f = d_xx rho)
        w1 = full_spectrum(plan) * vt + plan.c2 * lap_t + plan.A0 * vt
        out = dft.inverse(ds_symbol(plan) * w1, sign=-1, p=p).real / M
        if unpadded:       # transpose of f -> c2 Lap f composed with rho -> f
            out = out + plan.c2 * dft.inverse(ds_symbol(plan) * dft.forward(lap_v, sign=+1, p=p), sign=-1, p=p).real / M
        return out
    if plan.kernel != "dipolar3d":
        G = full_spectrum(plan)
        out = dft.inverse(G * vt, sign=-1, p=p).real / M
        if plan.A0 != 0.0 or plan.c2 != 0.0:
            lap = lap_v if unpadded else dft.inverse(lap_t, sign=-1, p=p).real / M
            out = out + plan.A0 * v + plan.c2 * lap
        return out
    nm = float(np.dot(plan.dipole_n, plan.dipole_m))
    G = full_spectrum(plan)
    sym = dipolar_symbol(plan)
    # transpose of rho -> -3 [I1 + A0 f + c2 Lap f](src(rho))
    w1 = G * vt + plan.c2 * lap_t + plan.A0 * vt
    out = dft.inverse(-sym * w1, sign=-1, p=p).real / M
    if unpadded:
        out = out + plan.c2 * dft.inverse(-sym * dft.forward(lap_v, sign=+1, p=p), sign=-1, p=p).real / M
    return -nm * v - 3.0 * out


def energy(plan: OraclePlan, rho: np.ndarray, u: np.ndarray | None = None) -> float:
    """Hartree-type energy 1/2 int rho u, by the grid (trapezoidal) sum."""
    if u is None:
        u = evaluate(plan, rho)
    return 0.5 * plan.cell * float(np.sum(rho * u))


def energy_gradient_rho(plan: OraclePlan, rho: np.ndarray) -> np.ndarray:
    """dE/drho = 1/2 h^d (A + A^T) rho."""
    return 0.5 * plan.cell * (evaluate(plan, rho) + adjoint(plan, rho))


def mixture_grid(n, L, a, mu, sigma):
    """rho = sum_c a_c exp(-|x - mu_c|^2 / sigma_c^2) on the grid x_j = -L + j h
    ([z][y][x] / [y][x] order, mu columns (x, y[, z]); n and L one value or one per
    axis in C order), with the per-component Gaussians g_c and squared distances
    r2_c and offsets x_i - mu_ci it is made of."""
    a = np.asarray(a, float)
    mu = np.asarray(mu, float)
    sigma = np.asarray(sigma, float)
    d = mu.shape[1]
    Ls = box_half_widths(L, d)
    ns = grid_points(n, d)
    axes = [-Lj + (2.0 * Lj / m) * np.arange(m) for Lj, m in zip(Ls, ns)]     # array-axis order
    if d == 3:
        X = (axes[2][None, None, :], axes[1][None, :, None], axes[0][:, None, None])   # x, y, z
    else:
        X = (axes[1][None, :], axes[0][:, None])
    shape = ns
    rho = np.zeros(shape)
    comps = []
    for c in range(len(a)):
        off = [np.broadcast_to(X[i] - mu[c, i], shape) for i in range(d)]
        r2 = sum(o * o for o in off)
        g = np.exp(-r2 / sigma[c] ** 2)
        rho += a[c] * g
        comps.append((g, r2, off))
    return rho, comps


def energy_gradient_params(plan: OraclePlan, a, mu, sigma):
    """E = 1/2 h^d sum rho u for the mixture density and its gradient with respect
    to (a, mu, sigma): dE/dtheta = sum_i (dE/drho_i) (drho_i/dtheta) with
      drho/da_c      = g_c
      drho/dmu_ci    = a_c g_c 2 (x_i - mu_ci) / sigma_c^2
      drho/dsigma_c  = a_c g_c 2 |x - mu_c|^2 / sigma_c^3.
    Returns (E, dE/da (K,), dE/dmu (K, d), dE/dsigma (K,))."""
    a = np.asarray(a, float)
    sigma = np.asarray(sigma, float)
    rho, comps = mixture_grid(plan.ns, plan.Ls, a, mu, sigma)
    gr = energy_gradient_rho(plan, rho)
    E = energy(plan, rho)
    K, d = len(a), plan.d
    ga, gmu, gs = np.zeros(K), np.zeros((K, d)), np.zeros(K)
    for c, (g, r2, off) in enumerate(comps):
        ga[c] = np.sum(gr * g)
        for i in range(d):
            gmu[c, i] = np.sum(gr * a[c] * g * 2.0 * off[i] / sigma[c] ** 2)
        gs[c] = np.sum(gr * a[c] * g * 2.0 * r2 / sigma[c] ** 3)
    return E, ga, gmu, gs
