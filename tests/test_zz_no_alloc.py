"""gs_eval_static: the evaluation with its workspace in the library's fixed device
array (no device allocation by the call), through the C ABI, against gs_eval's
output on the same plan (the same passes: bitwise equal) and against the oracle.

Two calls in a row, the second with a smaller input, so the second reuses the
array the first filled with a larger problem's intermediates."""

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_1501_04438_amd as gs
from paper_1501_04438_amd._lib import lib

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def static_eval(plan, rho):
    """gs_eval_static through the C ABI (ctypes), ordered on the current stream."""
    u = torch.empty_like(rho)
    plan._stream()
    st = lib().gs_eval_static(plan._h, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr()))
    assert st == 0, lib().gs_last_error().decode()
    return u


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("cases", [
    [("coulomb3d", 3, 128, 10.0, {}), ("coulomb3d", 3, 48, 6.0, {})],
    [("poisson2d", 2, 2048, 12.0, {"eps": 1e-13}), ("coulomb2d", 2, 96, 7.0, {})],
    [("dipolar3d", 3, 64, 8.0, {"dipole": ((0.3, -0.5, 0.8), (0.9, 0.1, -0.2))}),
     ("davey_stewartson2d", 2, 24, 6.0, {"eps": 1e-13})],
])
def test_static_equals_eval_two_calls(cases):
    for kernel, d, n, L, kw in cases:
        print(f"gs_eval_static: {kernel} d={d} n={n}", flush=True)
        rng = np.random.default_rng(900 + n)
        x = rng.standard_normal((n,) * d)
        plan = gs.Plan(kernel, n=n, L=L, d=d, **kw)
        rho = cuda(x)
        ref = plan.eval(rho)
        got = static_eval(plan, rho)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        if n <= 64:
            o = oracle.evaluate(oracle.make_plan(kernel, d, n, L, **kw), x)
            assert relmax(got.cpu().numpy(), o) <= TOL


def test_plan_without_workspace():
    """A plan created with GS_PLAN_NO_WORKSPACE holds no workspace: gs_eval refuses it,
    gs_eval_static evaluates it (bitwise as a plan with a workspace)."""
    n, L = 32, 5.0
    x = cuda(np.random.default_rng(5).standard_normal((n, n, n)))
    full = gs.Plan("coulomb3d", n=n, L=L)
    bare = gs.Plan("coulomb3d", n=n, L=L, workspace=False)
    assert bare.info["workspace_bytes"] < full.info["workspace_bytes"]
    with pytest.raises(gs.GSError):
        bare.eval(x)
    with pytest.raises(gs.GSError):
        gs.Batch([bare, full])
    got = static_eval(bare, x)
    ref = full.eval(x)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    # the slab layout: middle passes in kx slabs of 5 planes, X2 holding one slab
    sl = gs.Plan("coulomb3d", n=n, L=L, slab_planes=5, workspace=False)
    assert torch.equal(static_eval(sl, x), ref)


def test_oversized_workspace_is_refused():
    """A 3D plan at n = 192 needs 341 MB of workspace: beyond the 128 MiB array."""
    plan = gs.Plan("coulomb3d", n=192, L=8.0, workspace=False)
    x = torch.zeros((192,) * 3, dtype=torch.float64, device="cuda:0")
    u = torch.full_like(x, 7.0)
    st = lib().gs_eval_static(plan._h, C.c_void_p(x.data_ptr()), C.c_void_p(u.data_ptr()))
    assert st == 2                                            # GS_ERR_UNSUPPORTED_SIZE
    assert b"static scratch" in lib().gs_last_error()
    torch.cuda.synchronize()
    assert bool((u == 7.0).all())                             # outputs untouched
