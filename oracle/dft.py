"""Separable naive DFTs on the zero-padded grid (Section 2.2, eqs. (FourSeriB3), (rho_hat), (I1FFT)).

The density, sampled on n points per axis, is zero-padded to p n points (the box
[-p L, p L]; p = 2, the Remark after eq. (tensor), or p = 3, the box B_3 of
eq. (FourSeriB3)); its trapezoidal Fourier coefficients are then unnormalised
DFTs of length p n along every axis, in which only the n non-zero inputs take part:
    X[k] = sum_{j<n} x[j] exp(-2 pi i j k / (p n)),      k = 0..p n-1.
The inverse keeps the first n outputs (the original box):
    y[j] = sum_{k<p n} Y[k] exp(+2 pi i j k / (p n)),    j = 0..n-1.
The grid offset -L (and the padded box origin) adds a phase that cancels
between the forward and the inverse transform, so it is left out.

Each transform is a dense (n x p n) or (p n x n) matrix applied along one axis
with a BLAS matmul; phases use the exact integer reduction (j k) mod p n.
"""

from __future__ import annotations

import math
from functools import lru_cache

import numpy as np


@lru_cache(maxsize=16)
def _phase(n: int, sign: int, p: int = 2) -> np.ndarray:
    j = np.arange(n, dtype=np.int64)
    k = np.arange(p * n, dtype=np.int64)
    m = (j[:, None] * k[None, :]) % (p * n)
    ang = 2.0 * math.pi * m.astype(np.float64) / (p * n)
    return np.cos(ang) + sign * 1j * np.sin(ang)          # (n, p n): exp(sign * 2 pi i m / (p n))


def _apply_last(x: np.ndarray, mat: np.ndarray) -> np.ndarray:
    shp = x.shape
    y = np.ascontiguousarray(x).reshape(-1, shp[-1]) @ mat
    return y.reshape(shp[:-1] + (mat.shape[1],))


def _apply(x: np.ndarray, mat: np.ndarray, axis: int) -> np.ndarray:
    xt = np.moveaxis(x, axis, -1)
    return np.moveaxis(_apply_last(xt, mat), -1, axis)


def pad_dft(x: np.ndarray, axis: int, sign: int = -1, p: int = 2) -> np.ndarray:
    """Length-p n DFT of x zero-padded along `axis` (n -> p n)."""
    n = x.shape[axis]
    return _apply(x, _phase(n, sign, p), axis)


def crop_dft(X: np.ndarray, axis: int, sign: int = +1, p: int = 2) -> np.ndarray:
    """Length-p n DFT along `axis`, keeping the first n outputs (p n -> n)."""
    n = X.shape[axis] // p
    return _apply(X, _phase(n, sign, p).T, axis)


def forward(x: np.ndarray, sign: int = -1, p: int = 2) -> np.ndarray:
    X = x.astype(np.complex128)
    for ax in range(x.ndim - 1, -1, -1):
        X = pad_dft(X, ax, sign, p)
    return X


def inverse(X: np.ndarray, sign: int = +1, p: int = 2) -> np.ndarray:
    y = X
    for ax in range(X.ndim):
        y = crop_dft(y, ax, sign, p)
    return y


def full_dft(x: np.ndarray, sign: int = -1, p: int = 2) -> np.ndarray:
    """Non-separable O(M^2) DFT of the zero-padded array: brute force for tiny grids."""
    n = x.shape[0]
    d = x.ndim
    N = p * n
    idx = np.stack(np.meshgrid(*[np.arange(n)] * d, indexing="ij"), -1).reshape(-1, d)
    kdx = np.stack(np.meshgrid(*[np.arange(N)] * d, indexing="ij"), -1).reshape(-1, d)
    m = (kdx @ idx.T) % N
    mat = np.exp(sign * 2j * math.pi * m / N)
    return (mat @ x.reshape(-1)).reshape((N,) * d)


@lru_cache(maxsize=16)
def _periodic_phase(n: int, sign: int) -> np.ndarray:
    j = np.arange(n, dtype=np.int64)
    m = (j[:, None] * j[None, :]) % n
    ang = 2.0 * math.pi * m.astype(np.float64) / n
    return np.cos(ang) + sign * 1j * np.sin(ang)          # (n, n): exp(sign * 2 pi i m / n)


def periodic(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unpadded DFT of length n_j along every axis (the grid's own period), dense per axis."""
    X = x.astype(np.complex128)
    for ax in range(x.ndim):
        X = _apply(X, _periodic_phase(x.shape[ax], sign), ax)
    return X
