"""Gaussian-sum nonlocal potentials on AMD MI355X (Exl, Mauser, Zhang).

Python binding of the C ABI in include/gs.h.  Every step of an evaluation
runs in the HIP library libgs.so; this module only marshals arguments
(torch tensors give device pointers and the current stream).  Importing
works without a GPU; evaluating needs one, and fails loudly without the
built library.

    plan = Plan("coulomb3d", n=256, L=10.0, eps=1e-14)
    u = plan.eval(rho)                    # rho: (n, n, n) float64 CUDA tensor
    u = potential(rho, plan)              # autograd: backward runs the adjoint chain
    E = energy(rho, plan)                 # 1/2 h^d sum rho u
"""

from __future__ import annotations

import ctypes as C
import math

import numpy as np

from ._lib import (KERNEL_DIM, KERNELS, PLAN_AUTOTUNE, PLAN_HOST_ASSEMBLY, PLAN_HOST_ONLY, PLAN_NO_WORKSPACE,
                   PLAN_UNPADDED_LAPLACIAN, PLAN_PAD3, SCHEDULES, GSBatchInfo,
                   GSBatchOptions, GSError, GSOptions, GSPlanInfo, check, lib)

__all__ = ["Plan", "Batch", "SCHEDULES", "potential", "energy", "eval_batch", "GSError", "device_count", "supported_sizes",
           "mixture_density", "mixture_energy"]


def device_count() -> int:
    return int(lib().gs_device_count())


def supported_sizes(d: int) -> list[int]:
    buf = (C.c_int64 * 64)()
    c = lib().gs_supported_sizes(d, buf, 64)
    return [int(buf[i]) for i in range(min(c, 64))]


def _torch():
    import torch
    return torch


class Plan:
    """Precomputed state for one grid and kernel (Algorithm 1, precomputation).

    kernel: "coulomb3d" | "coulomb2d" | "poisson2d" | "dipolar3d" | "davey_stewartson2d" | "inverse_power"
            | "gaussian_sum" (the last two need d; "inverse_power" also beta: U = |x|^-beta, 0 < beta < d)
    n, L:   points per axis and box half-width: one value each for the cube [-L, L]^d with
            n^d points, or one per axis in array order ((nz, ny, nx), (Lz, Ly, Lx) / (ny, nx),
            (Ly, Lx)) for a rectangular box or grid (Section 2.5)
    eps:    Gaussian-sum accuracy; delta_rel: near-field radius / max L (below min L / max L)
    dipole: (n_vec, m_vec) for "dipolar3d"; custom: (w, tau) for "gaussian_sum"
    autotune: time the launch variants (cache hints per pass, fused-pass grid, tile shapes,
              the fused pass's radix plan) at plan creation and keep the fastest (cached per
              device and size; the results are bitwise the same for every variant but the
              radix plan, which agrees to rounding and is kept only when 1 % faster)
    tile_variants: tile shapes of the cubic passes and, bit 8, the fused pass's radix-plan
        variant (gs_options.tile_variants bits; 0 = defaults)
    hint_bits: cache-hint variants of the passes (bit p-1: pass p non-temporal; None = defaults)
    workspace: False creates the plan without an evaluation workspace of its own; it is
              then evaluated with eval_static only
    laplacian: "padded" (default) or "unpadded": the grid on which the near-field Taylor term
              takes the density's Laplacian (the padded grid of the convolution, or the
              density's own grid, periodic; kernels whose Taylor term acts on rho only)
    padding: 2 (default; the density zero-padded to [-2L, 2L]) or 3 (to B_3 = [-3L, 3L],
              Section 2.2; every n even, with 3n/2 a compiled transform length)
    """

    def __init__(self, kernel: str, n: int, L, eps: float = 1e-14, d: int | None = None,
                 delta_rel: float = 1e-4, dipole=None, custom=None, device: int = -1,
                 host_only: bool = False, host_assembly: bool = False, stream=None, slab_planes: int = 0,
                 slab_streams: int = 0, autotune: bool = False, beta: float | None = None,
                 workspace: bool = True, laplacian: str = "padded", tile_variants: int = 0,
                 padding: int = 2, hint_bits: int | None = None):
        if kernel not in KERNELS:
            raise ValueError(f"unknown kernel {kernel!r}")
        d = KERNEL_DIM.get(kernel, d)
        if d is None:
            raise ValueError(f"{kernel} plans need d")
        self.kernel, self.d, self.eps = kernel, int(d), float(eps)
        self.ns = _points(n, self.d)
        self.n = max(self.ns)
        self.Ls = _half_widths(L, self.d)
        self.L = max(self.Ls)
        self.padding = int(padding)
        opt = GSOptions()
        lib().gs_options_default(C.byref(opt))
        opt.delta_rel = float(delta_rel)
        opt.device = int(device)
        opt.flags = ((PLAN_HOST_ONLY if host_only else 0) | (PLAN_HOST_ASSEMBLY if host_assembly else 0)
                     | (PLAN_AUTOTUNE if autotune else 0) | (0 if workspace else PLAN_NO_WORKSPACE)
                     | (PLAN_UNPADDED_LAPLACIAN if laplacian == "unpadded" else 0)
                     | (PLAN_PAD3 if padding == 3 else 0))
        if laplacian not in ("padded", "unpadded"):
            raise ValueError("laplacian: padded or unpadded")
        if padding not in (2, 3):
            raise ValueError("padding: 2 or 3")
        opt.slab_planes = int(slab_planes)
        opt.tile_variants = int(tile_variants)
        if hint_bits is not None:
            opt.launch_hints = 1 + (int(hint_bits) & 31)
        opt.slab_streams = int(slab_streams)
        if beta is not None:
            opt.beta = float(beta)
        if stream is not None:
            opt.stream = C.c_void_p(int(stream))
        keep = []
        if dipole is not None:
            for i in range(3):
                opt.dipole_n[i] = float(dipole[0][i])
                opt.dipole_m[i] = float(dipole[1][i])
        if custom is not None:
            w = np.ascontiguousarray(custom[0], dtype=np.float64)
            tau = np.ascontiguousarray(custom[1], dtype=np.float64)
            keep += [w, tau]
            opt.gs_w = w.ctypes.data_as(C.POINTER(C.c_double))
            opt.gs_tau = tau.ctypes.data_as(C.POINTER(C.c_double))
            opt.gs_q = len(w)
        nn = (C.c_int64 * self.d)(*self.ns)
        LL = (C.c_double * self.d)(*self.Ls)
        h = C.c_void_p()
        check(lib().gs_plan_create(C.byref(h), KERNELS[kernel], self.d, nn, LL, self.eps, C.byref(opt)))
        self._h = h
        self.host_only = host_only
        self.info = self.query()

    # ------------------------------------------------------------- plan data
    def query(self) -> dict:
        info = GSPlanInfo()
        check(lib().gs_plan_query(self._h, C.byref(info)))
        out = {f: getattr(info, f) for f, _ in GSPlanInfo._fields_}
        out["L_axes"] = tuple(out["L_axes"][:self.d])
        out["n_axes"] = tuple(int(v) for v in out["n_axes"][:self.d])
        return out

    @property
    def h(self) -> float:
        """Grid step of a cubic box (`hs` holds the per-axis steps)."""
        hs = self.hs
        if len(set(hs)) > 1:
            raise ValueError("rectangular box: the grid step differs per axis")
        return hs[0]

    @property
    def hs(self) -> tuple:
        return tuple(2.0 * v / m for v, m in zip(self.Ls, self.ns))

    @property
    def cell(self) -> float:
        """Grid cell volume prod_j h_j."""
        return float(np.prod(self.hs))

    @property
    def shape(self):
        return tuple(self.ns)

    def table(self):
        Q = self.info["Q"]
        w, tau = np.empty(Q), np.empty(Q)
        check(lib().gs_plan_table(self._h, w.ctypes.data_as(C.POINTER(C.c_double)),
                                  tau.ctypes.data_as(C.POINTER(C.c_double)), Q))
        return w, tau

    def factors(self, axis: int | None = None) -> np.ndarray:
        """Factor matrix (p n / 2 + 1, Q) of array axis `axis` (default: the last, x), p the
        padding factor."""
        ax = self.d - 1 if axis is None else int(axis)
        F = np.empty((self.padding * self.ns[ax] // 2 + 1, self.info["Q"]))
        check(lib().gs_plan_factors_axis(self._h, ax, F.ctypes.data_as(C.POINTER(C.c_double)), F.size))
        return F

    def spectrum(self) -> np.ndarray:
        """The stored octant, indexed [kx][ky]([kz]) (x the first index), p n_j / 2 + 1 values
        per axis."""
        S = np.empty(tuple(self.padding * m // 2 + 1 for m in reversed(self.ns)))
        check(lib().gs_plan_spectrum(self._h, S.ctypes.data_as(C.POINTER(C.c_double)), S.size))
        return S

    # ------------------------------------------------------------- evaluation
    def _check_tensor(self, t, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != torch.float64 or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape {self.shape}")

    def _stream(self):
        torch = _torch()
        check(lib().gs_plan_set_stream(self._h, C.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def eval(self, rho, out=None):
        """u = U * rho on the grid (Algorithm 1, actual computation)."""
        torch = _torch()
        self._check_tensor(rho, "rho")
        u = torch.empty_like(rho) if out is None else out
        self._check_tensor(u, "out")
        self._stream()
        check(lib().gs_eval(self._h, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr())))
        return u

    def eval_static(self, rho, out=None):
        """As eval, with the workspace in the library's fixed device array (no device
        allocation by the library; calls on one device must not overlap in time)."""
        torch = _torch()
        self._check_tensor(rho, "rho")
        u = torch.empty_like(rho) if out is None else out
        self._check_tensor(u, "out")
        self._stream()
        check(lib().gs_eval_static(self._h, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr())))
        return u

    def mixture_density(self, a, mu, sigma, out=None):
        """rho = sum_c a_c exp(-|x - mu_c|^2 / sigma_c^2) on the plan's grid (a, sigma: (K,), mu: (K, d)
        with columns (x, y[, z]); float64 device tensors), formed by the library."""
        torch = _torch()
        a, mu, sigma = (t.detach().contiguous() for t in (a, mu, sigma))
        rho = torch.empty(self.shape, dtype=torch.float64, device=a.device) if out is None else out
        self._check_tensor(rho, "out")
        self._stream()
        check(lib().gs_mixture_density(self._h, int(a.numel()), C.c_void_p(a.data_ptr()), C.c_void_p(mu.data_ptr()),
                                       C.c_void_p(sigma.data_ptr()), C.c_void_p(rho.data_ptr())))
        return rho

    def mixture_gradient(self, a, mu, sigma, g, scale: float = 1.0, flat: bool = False):
        """(d/da, d/dmu, d/dsigma) of a scalar whose grid gradient is scale * g, through the mixture
        density (the library's fixed-order reduction); flat: the K (d + 2) values in one tensor."""
        torch = _torch()
        a, mu, sigma = (t.detach().contiguous() for t in (a, mu, sigma))
        self._check_tensor(g, "g")
        K, d = int(a.numel()), self.d
        out = torch.empty(K * (d + 2), dtype=torch.float64, device=a.device)
        self._stream()
        check(lib().gs_mixture_gradient(self._h, K, C.c_void_p(a.data_ptr()), C.c_void_p(mu.data_ptr()),
                                        C.c_void_p(sigma.data_ptr()), C.c_void_p(g.data_ptr()), float(scale),
                                        C.c_void_p(out.data_ptr())))
        if flat:
            return out
        return out[:K], out[K:K + K * d].view(K, d), out[K + K * d:]

    def eval_energy(self, rho, out=None):
        """(u, E): the potential and E = 1/2 cell sum rho u (a 0-d device tensor), the sum
        formed in the fused spectrum pass (Parseval's identity) and totalled in a fixed order."""
        torch = _torch()
        self._check_tensor(rho, "rho")
        u = torch.empty_like(rho) if out is None else out
        self._check_tensor(u, "out")
        E = torch.empty((), dtype=torch.float64, device=rho.device)
        self._stream()
        check(lib().gs_eval_energy(self._h, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr()),
                                   C.c_void_p(E.data_ptr())))
        return u, E

    def energy_and_gradient(self, rho, out=None):
        """(E, dE/drho) of E = 1/2 cell sum rho u without autograd: one evaluation whose last
        pass writes the gradient cell * u, the energy summed as in eval_energy (a 0-d device
        tensor)."""
        torch = _torch()
        self._check_tensor(rho, "rho")
        g = torch.empty_like(rho) if out is None else out
        self._check_tensor(g, "out")
        E = torch.empty((), dtype=torch.float64, device=rho.device)
        self._stream()
        check(lib().gs_eval_energy_gradient(self._h, C.c_void_p(rho.data_ptr()), C.c_void_p(g.data_ptr()),
                                            C.c_void_p(E.data_ptr())))
        return E, g

    def eval_backward(self, grad_u, out=None):
        """grad_rho = A^T grad_u (the transposed chain)."""
        torch = _torch()
        self._check_tensor(grad_u, "grad_u")
        g = torch.empty_like(grad_u) if out is None else out
        self._check_tensor(g, "out")
        self._stream()
        check(lib().gs_eval_backward(self._h, C.c_void_p(grad_u.data_ptr()), C.c_void_p(g.data_ptr())))
        return g

    def steps(self) -> list[int]:
        """Pass id of every kernel launch of one evaluation, in order."""
        c = lib().gs_plan_steps(self._h, None, 0)
        buf = (C.c_int * max(c, 1))()
        lib().gs_plan_steps(self._h, buf, c)
        return [int(buf[i]) for i in range(c)]

    def eval_step(self, rho, u, step: int):
        self._stream()
        check(lib().gs_eval_step(self._h, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr()), int(step)))

    def eval_events(self, rho, u, events):
        """eval with the given HIP event handles (steps + 1) recorded around every step (None: no record)."""
        self._stream()
        arr = (C.c_void_p * len(events))(*[e.value if hasattr(e, "value") else e for e in events])
        check(lib().gs_eval_events(self._h, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr()), arr, len(events)))

    def eval_pass(self, rho, u, p: int):
        """Run every step of pass p (1..5) in order (one slab plans: the pass itself)."""
        for i, q in enumerate(self.steps()):
            if q == p:
                self.eval_step(rho, u, i)

    def buffer(self, which: int, value=None):
        """Read (value None) or write a plan buffer: 1 = X1, 2 = X2 (complex), 3 = spectrum."""
        d = self.d
        nx, ny = self.ns[-1], self.ns[-2]
        nz = self.ns[0] if d == 3 else 1
        if which == 1:
            shape, cplx = ((nz, nx + 1, ny) if d == 3 else (nx + 1, ny)), True
        elif which == 2:
            shape, cplx = (self.query()["x2_planes"], 2 * ny, nz), True
        else:
            shape, cplx = tuple(m + 1 for m in reversed(self.ns)), False
        if value is None:
            a = np.empty(shape, np.complex128 if cplx else np.float64)
            check(lib().gs_plan_buffer(self._h, which, 0, a.ctypes.data_as(C.POINTER(C.c_double)),
                                       a.size * (2 if cplx else 1)))
            return a
        a = np.ascontiguousarray(value, np.complex128 if cplx else np.float64).reshape(shape)
        check(lib().gs_plan_buffer(self._h, which, 1, a.ctypes.data_as(C.POINTER(C.c_double)),
                                   a.size * (2 if cplx else 1)))

    def close(self):
        if getattr(self, "_h", None):
            lib().gs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_batch(plans, rhos, outs=None):
    """Evaluate independent problems (one plan each) in one batched launch."""
    torch = _torch()
    if outs is None:
        outs = [torch.empty_like(r) for r in rhos]
    for p, r, o in zip(plans, rhos, outs):
        p._check_tensor(r, "rho")
        p._check_tensor(o, "out")
    n = len(plans)
    hs = (C.c_void_p * n)(*[p._h for p in plans])
    rs = (C.c_void_p * n)(*[r.data_ptr() for r in rhos])
    us = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    plans[0]._stream()
    check(lib().gs_eval_batch(n, hs, rs, us))
    return outs


class Batch:
    """Many independent problems (one plan each, sizes may differ) evaluated together.

    schedule: "auto" (measured on the first eval, cached; GS_AUTOTUNE_CACHE names a
    JSON file to keep it across processes), "queue" (one persistent launch),
    "phased" (one launch per pass type), "sized" (one launch per pass type and grid
    size), "concurrent" (the sized launches, each grid size's chain on its own stream),
    "sequential" (each plan's own eval) or "streams" (each plan's own eval, the plans
    dealt to four concurrent streams).
    graph=True captures the launch sequence in a hipGraph and replays it.
    Every schedule gives each problem bitwise the result of plan.eval.
    """

    def __init__(self, plans, schedule: str = "auto", graph: bool = False, tiles_per_task: int = 0,
                 grid: int = 0):
        torch = _torch()
        self.plans = list(plans)
        opt = GSBatchOptions()
        lib().gs_batch_options_default(C.byref(opt))
        opt.schedule = SCHEDULES[schedule]
        opt.tiles_per_task = int(tiles_per_task)
        opt.grid = int(grid)
        opt.use_graph = 1 if graph else 0
        opt.stream = torch.cuda.current_stream().cuda_stream
        n = len(self.plans)
        hs = (C.c_void_p * n)(*[p._h for p in self.plans])
        h = C.c_void_p()
        check(lib().gs_batch_create(C.byref(h), n, hs, C.byref(opt)))
        self._h = h

    def eval(self, rhos, outs=None):
        torch = _torch()
        if outs is None:
            outs = [torch.empty_like(r) for r in rhos]
        if len(rhos) != len(self.plans) or len(outs) != len(self.plans):
            raise ValueError("one rho and one out per plan")
        for p, r, o in zip(self.plans, rhos, outs):
            p._check_tensor(r, "rho")
            p._check_tensor(o, "out")
        n = len(self.plans)
        rs = (C.c_void_p * n)(*[r.data_ptr() for r in rhos])
        us = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        # ordered after the stream current at this call (as Plan.eval is)
        check(lib().gs_batch_set_stream(self._h, C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        check(lib().gs_batch_eval(self._h, rs, us))
        return outs

    @property
    def info(self) -> dict:
        i = GSBatchInfo()
        check(lib().gs_batch_query(self._h, C.byref(i)))
        names = {v: k for k, v in SCHEDULES.items()}
        out = {f: getattr(i, f) for f, _ in GSBatchInfo._fields_ if f != "tasks_per_pass"}
        out["schedule"] = names[out["schedule"]]
        out["tasks_per_pass"] = [int(i.tasks_per_pass[p]) for p in range(6)]
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().gs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ autograd

def _make_function():
    torch = _torch()

    class GSPotential(torch.autograd.Function):
        """u = A rho with A the discrete Gaussian-sum convolution; backward applies A^T."""

        @staticmethod
        def forward(ctx, rho, plan):
            ctx.plan = plan
            return plan.eval(rho.contiguous())

        @staticmethod
        def backward(ctx, grad_u):
            return ctx.plan.eval_backward(grad_u.contiguous()), None

    class GSEnergy(torch.autograd.Function):
        """E = 1/2 cell sum rho (A rho).  A is symmetric (the spectrum is real and even, and the
        zero padding and the cropping are transposes of each other; the library's transposed
        chain is the forward chain), so dE/drho = cell A rho = cell u: the backward reuses the
        forward's potential instead of running the adjoint solve."""

        @staticmethod
        def forward(ctx, rho, plan):
            rho = rho.contiguous()
            u, E = plan.eval_energy(rho)
            ctx.save_for_backward(u)
            ctx.cell = plan.cell
            return E

        @staticmethod
        def backward(ctx, grad_e):
            (u,) = ctx.saved_tensors
            return (grad_e * ctx.cell) * u, None

    class GSMixtureEnergy(torch.autograd.Function):
        """E(a, mu, sigma) = 1/2 cell sum rho u for the Gaussian-mixture density: the density, the
        evaluation with its energy and the parameter gradient (cell u through the density's
        derivatives) all run in the library."""

        @staticmethod
        def forward(ctx, a, mu, sigma, plan):
            rho = plan.mixture_density(a, mu, sigma)
            u, E = plan.eval_energy(rho, out=rho)
            ctx.save_for_backward(a, mu, sigma, u)
            ctx.plan = plan
            return E

        @staticmethod
        def backward(ctx, grad_e):
            a, mu, sigma, u = ctx.saved_tensors
            # the three gradients in one buffer: one product scales them all
            out = ctx.plan.mixture_gradient(a, mu, sigma, u, ctx.plan.cell, flat=True) * grad_e
            K, d = a.numel(), ctx.plan.d
            return out[:K], out[K:K + K * d].view(K, d), out[K + K * d:], None

    return GSPotential, GSEnergy, GSMixtureEnergy


_FUNCS = None


def _functions():
    global _FUNCS
    if _FUNCS is None:
        _FUNCS = _make_function()
    return _FUNCS


def potential(rho, plan: Plan):
    """u = U * rho as a differentiable function of rho (backward: the adjoint solve)."""
    return _functions()[0].apply(rho, plan)


def energy(rho, plan: Plan):
    """Hartree-type energy E = 1/2 int rho u, by the grid sum 1/2 (prod_j h_j) sum rho u;
    differentiable in rho with one solve (dE/drho = prod_j h_j u, the operator being symmetric)."""
    return _functions()[1].apply(rho, plan)


def mixture_energy(a, mu, sigma, plan: Plan):
    """Energy 1/2 int rho u of the Gaussian mixture rho = sum_c a_c exp(-|x - mu_c|^2/sigma_c^2)
    on the plan's grid, differentiable in (a, mu, sigma): the density, the evaluation with
    its energy, and the gradient's reduction run in the library (one solve)."""
    return _functions()[2].apply(a, mu, sigma, plan)


def _points(n, d: int) -> tuple:
    if np.ndim(n) == 0:
        return (int(n),) * d
    ns = tuple(int(v) for v in n)
    if len(ns) != d:
        raise ValueError("n: one value, or one per axis")
    return ns


def _half_widths(L, d: int) -> tuple:
    if np.ndim(L) == 0:
        return (float(L),) * d
    Ls = tuple(float(v) for v in L)
    if len(Ls) != d:
        raise ValueError("L: one half-width, or one per axis")
    return Ls


def mixture_density(a, mu, sigma, n, L):
    """Gaussian mixture sum_c a_c exp(-|x - mu_c|^2/sigma_c^2) on the [z][y][x] grid as a
    differentiable torch expression (input construction for parameter gradients).
    n, L: one value or one per axis in array order."""
    torch = _torch()
    d = mu.shape[1]
    Ls = _half_widths(L, d)
    ns = _points(n, d)
    ax = [-Lj + (2.0 * Lj / m) * torch.arange(m, dtype=torch.float64, device=mu.device) for Lj, m in zip(Ls, ns)]
    if d == 3:
        X = (ax[2].view(1, 1, -1), ax[1].view(1, -1, 1), ax[0].view(-1, 1, 1))
    else:
        X = (ax[1].view(1, -1), ax[0].view(-1, 1))
    out = 0.0
    for c in range(mu.shape[0]):
        r2 = sum((X[i] - mu[c, i]) ** 2 for i in range(d))
        out = out + a[c] * torch.exp(-r2 / sigma[c] ** 2)
    return out
