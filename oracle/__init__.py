"""Oracle for the Gaussian-sum potential evaluation (Exl, Mauser, Zhang).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 CPU
implementation of the method, written from the paper: the Gaussian-sum table
from sinc quadrature (Section 3), the one-dimensional factor integrals of the
tensor-product kernel coefficients (Section 2.2, eq. (tensor)), the zero-padded
trigonometric (trapezoidal) Fourier coefficients of the density (eqs.
(FourSeriB3), (rho_hat)), the regular integral by the inverse transform (eq. (I1FFT)), and
the Taylor near-field correction (Section 2.3, eq. (taylor)), summed as in
Algorithm 1.  Transforms are separable naive DFTs (dense per-axis DFT matrices
applied by a BLAS matmul); there is no FFT factorisation anywhere.

It shares no code with the GPU library under ``paper_1501_04438_amd`` and
imports nothing from it.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.

Every numerical choice the paper leaves open is fixed here by a documented
reading (grid offset, padding factor 2, fit interval [delta, 2*sqrt(d)],
delta = 1e-4 in box units, Laplacian on the padded grid, Nyquist handling).
"""

from .gs_table import coulomb_table, poisson_table, physical_table, GSTable
from .factors import factor_1d
from .taylor import taylor_constants
from .evaluate import (OraclePlan, make_plan, evaluate, adjoint, energy,
                       energy_gradient_rho, energy_gradient_params, mixture_grid,
                       full_spectrum, padded_frequencies, laplacian_symbol, dipolar_symbol)
from . import closed_forms, dft

__all__ = [
    "coulomb_table", "poisson_table", "physical_table", "GSTable", "factor_1d",
    "taylor_constants", "OraclePlan", "make_plan", "evaluate", "adjoint", "energy",
    "energy_gradient_rho", "energy_gradient_params", "mixture_grid", "full_spectrum", "padded_frequencies",
    "laplacian_symbol", "dipolar_symbol", "closed_forms", "dft",
]
