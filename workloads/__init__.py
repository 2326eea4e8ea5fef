"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random parameters and samples densities on grids.  It
holds none of the potential-evaluation arithmetic: neither the oracle nor the
GPU library imports anything from here, and nothing here imports either of them.

Grid convention (one axis): ``x_j = -L + j*h`` with ``h = 2L/n`` and
``j = 0..n-1``.  Arrays are C-ordered ``[z][y][x]`` (3D) or ``[y][x]`` (2D), with
x the last, fastest-varying index.

Workloads follow the experiments of the paper (Section 4): Gaussian densities,
shifted and anisotropic Gaussians, and Gaussian mixtures on cubic boxes, and
anisotropic Gaussians on rectangular boxes (one half-width per axis, given in
C order: ``(Lz, Ly, Lx)`` in 3D, ``(Ly, Lx)`` in 2D; n points on every axis).
Random draws use ``numpy.random.default_rng(150104438 + config_id)``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 150104438

# Dipole orientations printed with the dipolar example (Section 4, Example 4.4).
PAPER_DIPOLE_N = (0.82778, 0.41505, -0.37751)
PAPER_DIPOLE_M = (0.3118, 0.9378, -0.15214)


def axis(n: int, L: float) -> np.ndarray:
    """Grid points of one axis: ``-L + j*2L/n`` for ``j = 0..n-1``."""
    return -L + (2.0 * L / n) * np.arange(n, dtype=np.float64)


def half_widths(L, d: int) -> tuple:
    """``(L,)*d`` for a cube, else the given per-axis half-widths (C order)."""
    if np.ndim(L) == 0:
        return (float(L),) * d
    Ls = tuple(float(v) for v in L)
    if len(Ls) != d:
        raise ValueError("one half-width per axis")
    return Ls


def points(n, d: int) -> tuple:
    """``(n,)*d`` for one value, else the given per-axis points (C order)."""
    if np.ndim(n) == 0:
        return (int(n),) * d
    ns = tuple(int(v) for v in n)
    if len(ns) != d:
        raise ValueError("one n per axis")
    return ns


def mesh(n, L, d: int):
    """Coordinate arrays (x, y[, z]) broadcastable to the ``[z][y][x]`` grid (n and L one
    value or one per axis in C order)."""
    if d not in (2, 3):
        raise ValueError("d must be 2 or 3")
    Ls = half_widths(L, d)
    ns = points(n, d)
    if d == 2:
        return axis(ns[1], Ls[1])[None, :], axis(ns[0], Ls[0])[:, None]
    return (axis(ns[2], Ls[2])[None, None, :], axis(ns[1], Ls[1])[None, :, None],
            axis(ns[0], Ls[0])[:, None, None])


@dataclass
class Mixture:
    """Gaussian mixture ``rho(x) = sum_c a_c exp(-|x - mu_c|^2 / sigma_c^2)``."""

    a: np.ndarray        # (K,)
    mu: np.ndarray       # (K, d), columns ordered (x, y[, z])
    sigma: np.ndarray    # (K,)

    @property
    def d(self) -> int:
        return self.mu.shape[1]


def draw_mixture(rng: np.random.Generator, K: int, d: int, mu_range: float = 2.0,
                 sigma_range=(0.5, 2.0)) -> Mixture:
    """Draw sigma ~ U[0.5, 2], a ~ U(-1, 1), mu ~ U[-2, 2]^d, in that order."""
    sigma = rng.uniform(sigma_range[0], sigma_range[1], K)
    a = rng.uniform(-1.0, 1.0, K)
    mu = rng.uniform(-mu_range, mu_range, (K, d))
    return Mixture(a=a, mu=mu, sigma=sigma)


def sample_mixture(m: Mixture, n: int, L: float) -> np.ndarray:
    """Each component is a product of one-dimensional Gaussians (outer products)."""
    d = m.d
    ax = axis(n, L)
    out = np.zeros((n,) * d)
    for c in range(len(m.a)):
        f = [np.exp(-((ax - m.mu[c, i]) ** 2) / m.sigma[c] ** 2) for i in range(d)]   # (x, y[, z])
        if d == 3:
            out += m.a[c] * (f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :])
        else:
            out += m.a[c] * (f[1][:, None] * f[0][None, :])
    return out


def gaussian(n, L, d: int, sigma: float = 1.0, center=None,
             gammas=None, scale: float = 1.0) -> np.ndarray:
    """``scale * exp(-sum_i gamma_i^2 (x_i - c_i)^2 / sigma^2)`` on the grid
    (center and gammas in (x, y[, z]) order; n and L scalar or per axis in C order)."""
    Ls = half_widths(L, d)
    ns = points(n, d)
    center = np.zeros(d) if center is None else np.asarray(center, float)
    gammas = np.ones(d) if gammas is None else np.asarray(gammas, float)
    f = [np.exp(-((gammas[i] * (axis(ns[d - 1 - i], Ls[d - 1 - i]) - center[i])) ** 2) / sigma ** 2)
         for i in range(d)]
    if d == 3:
        return scale * (f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :])
    return scale * (f[1][:, None] * f[0][None, :])


# --------------------------------------------------------------------------
# The benchmark configurations.
# --------------------------------------------------------------------------

@dataclass
class Problem:
    kernel: str          # "coulomb3d" | "coulomb2d" | "poisson2d" | "dipolar3d"
    d: int
    n: int
    L: float             # half-width of the cube, or per-axis half-widths (C order)
    rho: np.ndarray
    mixture: Mixture | None = None
    extra: dict = field(default_factory=dict)


def config1(n: int = 32) -> Problem:
    """3D Coulomb, normalised isotropic Gaussian exp(-|x|^2)/pi^(3/2) on [-8,8]^3."""
    rho = gaussian(n, 8.0, 3, sigma=1.0, scale=math.pi ** -1.5)
    return Problem("coulomb3d", 3, n, 8.0, rho)


def config2_mixture() -> Mixture:
    rng = np.random.default_rng(SEED_BASE + 2)
    return draw_mixture(rng, 8, 3)


def config2(n: int = 256) -> Problem:
    """3D Coulomb on [-10,10]^3: triaxial Gaussian exp(-(x^2+4y^2+16z^2)) plus an
    8-component seeded mixture (sigma in [0.5,2], a in (-1,1), mu in [-2,2]^3)."""
    L = 10.0
    mix = config2_mixture()
    rho = gaussian(n, L, 3, sigma=1.0, gammas=(1.0, 2.0, 4.0)) + sample_mixture(mix, n, L)
    return Problem("coulomb3d", 3, n, L, rho, mixture=mix,
                   extra={"triaxial_a": (1.0, 4.0, 16.0)})


def config3_mixture() -> Mixture:
    rng = np.random.default_rng(SEED_BASE + 3)
    return draw_mixture(rng, 16, 2)


def config3_2d(kernel: str, n: int = 1024) -> Problem:
    """2D Poisson, 2D Coulomb or Davey-Stewartson potential of a seeded 16-Gaussian
    mixture on [-12,12]^2."""
    assert kernel in ("poisson2d", "coulomb2d", "davey_stewartson2d")
    L = 12.0
    mix = config3_mixture()
    return Problem(kernel, 2, n, L, sample_mixture(mix, n, L), mixture=mix)


def config3_dipoles():
    """Seeded unit dipole orientations (normalised standard-normal draws)."""
    rng = np.random.default_rng(SEED_BASE + 33)
    v = rng.standard_normal((2, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return tuple(v[0]), tuple(v[1])


def config3_dipolar(n: int = 128, paper_vectors: bool = False) -> Problem:
    """3D dipolar potential of exp(-|x|^2/1.44) on [-8,8]^3 (the density of the
    dipolar example, sigma = 1.2)."""
    if paper_vectors:
        dn, dm = PAPER_DIPOLE_N, PAPER_DIPOLE_M
    else:
        dn, dm = config3_dipoles()
    rho = gaussian(n, 8.0, 3, sigma=1.2)
    return Problem("dipolar3d", 3, n, 8.0, rho, extra={"n": dn, "m": dm, "sigma": 1.2})


def rect_box(d: int, gamma: float, n: int | None = None) -> Problem:
    """Anisotropic examples of Section 4 on rectangular boxes: sigma = 2 and
      3D Coulomb, exp(-(x^2 + y^2 + gamma^2 z^2)/sigma^2) on [-12,12]^2 x [-12,12]/gamma,
         n = 96 per axis (h_x = h_y = 1/4, h_z = h_x/gamma; Table 3);
      2D Coulomb, exp(-(x^2 + gamma^2 y^2)/sigma^2) on [-12,12] x [-12,12]/gamma,
         n = 192 per axis (h_x = 1/8, h_y = h_x/gamma; Table 5)."""
    if d == 3:
        n = 96 if n is None else n
        Ls = (12.0 / gamma, 12.0, 12.0)
        rho = gaussian(n, Ls, 3, sigma=2.0, gammas=(1.0, 1.0, gamma))
        return Problem("coulomb3d", 3, n, Ls, rho, extra={"sigma": 2.0, "gamma": gamma})
    n = 192 if n is None else n
    Ls = (12.0 / gamma, 12.0)
    rho = gaussian(n, Ls, 2, sigma=2.0, gammas=(1.0, gamma))
    return Problem("coulomb2d", 2, n, Ls, rho, extra={"sigma": 2.0, "gamma": gamma})


def ds_example(n: int = 256) -> Problem:
    """Davey-Stewartson example (Example 4.5): rho = pi exp(-pi^2 |x|^2) on [-8,8]^2."""
    rho = gaussian(n, 8.0, 2, sigma=1.0 / math.pi, scale=math.pi)
    return Problem("davey_stewartson2d", 2, n, 8.0, rho)


BATCH_SIZES = (32, 48, 64, 96, 128)


def config4(count: int = 64) -> list[Problem]:
    """Batch of seeded mixtures (4..32 components) on grids drawn from
    {32,48,64,96,128}^3, box [-10,10]^3, 3D Coulomb."""
    rng = np.random.default_rng(SEED_BASE + 4)
    out = []
    for _ in range(count):
        n = int(rng.choice(BATCH_SIZES))
        K = int(rng.integers(4, 33))
        mix = draw_mixture(rng, K, 3)
        out.append(Problem("coulomb3d", 3, n, 10.0, None, mixture=mix))
    return out


def materialise(p: Problem) -> Problem:
    if p.rho is None:
        p.rho = sample_mixture(p.mixture, p.n, p.L)
    return p


def config5_mixture() -> Mixture:
    """The 8-component mixture of the differentiation workload (same draws as
    the headline mixture, without the triaxial term)."""
    return config2_mixture()


def config5(n: int = 256) -> Problem:
    L = 10.0
    mix = config5_mixture()
    return Problem("coulomb3d", 3, n, L, sample_mixture(mix, n, L), mixture=mix)


def random_field(rng: np.random.Generator, shape, smooth: bool = False) -> np.ndarray:
    """Plain random grid data for operator-level checks (linearity, adjoint)."""
    return rng.standard_normal(shape)
