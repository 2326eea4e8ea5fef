"""The C ABI: the library loads, exports every function include/gs.h declares,
and validates arguments on the host (no device is touched by these tests)."""

import ctypes as C
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import paper_1501_04438_amd as gs
from paper_1501_04438_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "gs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported_and_bound():
    L = _lib.lib()
    names = header_functions()
    assert "gs_eval" in names and "gs_plan_create" in names and "gs_eval_batch" in names
    for name in names:
        assert hasattr(L, name), name
        assert name in _lib.SIGNATURES, name


def test_nm_exports_c_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (gs_[a-z_]+)\b", out))
    assert set(header_functions()) <= exported


def _create(kernel=0, d=3, n=16, L=4.0, eps=1e-14, flags=_lib.PLAN_HOST_ONLY, nlist=None, **kw):
    opt = _lib.GSOptions()
    _lib.lib().gs_options_default(C.byref(opt))
    opt.flags = flags
    for k, v in kw.items():
        setattr(opt, k, v)
    h = C.c_void_p()
    nn = (C.c_int64 * d)(*(nlist if nlist is not None else [n] * d))
    LL = (C.c_double * d)(*(L if isinstance(L, (tuple, list)) else [L] * d))
    st = _lib.lib().gs_plan_create(C.byref(h), kernel, d, nn, LL, eps, C.byref(opt))
    return st, h


def test_argument_validation_statuses():
    ok, h = _create()
    assert ok == 0
    assert _lib.lib().gs_plan_destroy(h) == 0
    assert _lib.lib().gs_plan_destroy(h) == 0            # idempotent per handle
    assert _lib.lib().gs_plan_destroy(None) == 0         # NULL is a no-op
    assert _create(d=4)[0] == 1
    assert _create(kernel=0, d=2)[0] == 1                # kernel/dimension disagree
    assert _create(kernel=9)[0] == 1
    assert _create(L=-1.0)[0] == 1
    assert _create(eps=0.0)[0] == 1
    assert _create(n=22)[0] == 2                         # no kernels for n = 22 (a factor 11)
    assert _create(n=4096)[0] == 2
    assert _create(eps=1e-20)[0] == 3                    # below the table floor
    assert _create(kernel=2, d=2, eps=1e-15)[0] == 3     # ln-table rounding floor
    assert _create(kernel=3, d=3)[0] == 1                # dipole vectors must be non-zero
    assert _create(kernel=4, d=3)[0] == 1                # custom sum missing
    msg = _lib.lib().gs_last_error().decode()
    assert "custom" in msg
    assert _create(kernel=6, d=3)[0] == 1                # inverse power without beta
    assert _create(kernel=6, d=2, beta=2.0)[0] == 1      # beta must be below d
    st, h = _create(kernel=6, d=3, beta=1.5)
    assert st == 0 and _lib.lib().gs_plan_destroy(h) == 0
    assert _create(nlist=[16, 22, 32])[0] == 2           # every axis' n must be compiled
    assert "n = 22" in _lib.lib().gs_last_error().decode()
    assert _create(nlist=[16, 1, 32])[0] == 1            # and at least 2
    assert _create(L=(4.0, 4.0, -1.0))[0] == 1
    assert _create(L=(1e-4, 4.0, 4.0))[0] == 1           # near-field ball wider than the short axis
    assert "shortest" in _lib.lib().gs_last_error().decode()
    st, h = _create(L=(1.0, 2.0, 4.0))                   # rectangular box
    assert st == 0
    info = _lib.GSPlanInfo()
    assert _lib.lib().gs_plan_query(h, C.byref(info)) == 0
    assert info.L == 4.0 and tuple(info.L_axes) == (1.0, 2.0, 4.0)
    F = (C.c_double * (17 * info.Q))()
    assert _lib.lib().gs_plan_factors_axis(h, 3, F, len(F)) == 1
    assert _lib.lib().gs_plan_factors_axis(h, 0, F, len(F)) == 0
    assert _lib.lib().gs_plan_destroy(h) == 0
    st, h = _create(nlist=[16, 24, 32], L=(2.0, 3.0, 4.0))   # one n per axis
    assert st == 0
    assert _lib.lib().gs_plan_query(h, C.byref(info)) == 0
    assert tuple(info.n_axes) == (16, 24, 32) and info.n == 32
    assert _lib.lib().gs_plan_factors_axis(h, 1, F, len(F)) == 1     # 25 rows: capacity 17 Q too small
    F25 = (C.c_double * (25 * info.Q))()
    assert _lib.lib().gs_plan_factors_axis(h, 1, F25, len(F25)) == 0
    assert _lib.lib().gs_plan_destroy(h) == 0


def test_no_device_and_workspace_cap():
    # a device plan on a machine without a GPU reports NO_DEVICE; the workspace cap
    # is checked first and forced with GS_MAX_WORKSPACE_BYTES=0
    code = ("import ctypes as C, os, sys; sys.path.insert(0, %r);"
            "from paper_1501_04438_amd import _lib;"
            "o=_lib.GSOptions(); _lib.lib().gs_options_default(C.byref(o)); h=C.c_void_p();"
            "n=(C.c_int64*3)(16,16,16); L=(C.c_double*3)(4.,4.,4.);"
            "print(_lib.lib().gs_plan_create(C.byref(h),0,3,n,L,1e-14,C.byref(o)))") % ROOT
    env = dict(os.environ, GS_MAX_WORKSPACE_BYTES="0")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env)
    assert r.stdout.strip() == "4", r.stderr
    if gs.device_count() == 0:
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
        assert r.stdout.strip() == "5", r.stderr


def test_host_only_plan_refuses_evaluation():
    st, h = _create()
    assert st == 0
    L = _lib.lib()
    assert L.gs_eval(h, C.c_void_p(16), C.c_void_p(16)) == 1
    assert L.gs_eval_backward(h, C.c_void_p(16), C.c_void_p(16)) == 1
    assert L.gs_eval_step(h, C.c_void_p(16), C.c_void_p(16), 3) == 1
    assert L.gs_eval_events(h, C.c_void_p(16), C.c_void_p(16), None, 6) == 1
    assert L.gs_plan_steps(h, None, 0) == 5          # 3D: x, (y, fused, y) for one slab, x
    arr = (C.c_void_p * 1)(h.value)
    assert L.gs_eval_batch(1, arr, arr, arr) == 1
    assert L.gs_eval_batch(0, arr, arr, arr) == 1
    L.gs_plan_destroy(h)


def test_status_strings_and_sizes():
    L = _lib.lib()
    for s, name in _lib.STATUS.items():
        assert L.gs_status_string(s).decode() == name
    s3, s2 = gs.supported_sizes(3), gs.supported_sizes(2)
    assert 256 in s3 and 2048 not in s3 and 2048 in s2 and s3 == sorted(s3)
    # 5-smooth and 7-smooth lengths (radix-5 and radix-7 stages)
    assert {20, 40, 80, 160, 320, 640, 28, 56, 112, 224} <= set(s3)


def test_plan_query_fields():
    p = gs.Plan("coulomb3d", n=32, L=8.0, host_only=True)
    i = p.info
    assert i["S"] == 248 and i["Q"] == 249 and i["host_only"] == 1
    assert abs(i["delta"] - 8.0e-4) < 1e-18
    assert i["spectrum_bytes"] == 33 ** 3 * 8
    assert i["workspace_bytes"] == (33 * 32 * 32 + 2 * 32 * 32 * 33) * 16 + 64 * 16
