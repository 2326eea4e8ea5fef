"""Each evaluation pass on its own, against a NumPy DFT of the same layout.

The plan's workspace is filled from the host (gs_plan_buffer), one pass runs
(gs_eval_step on a one-slab plan), and its output is read back.  Layouts (complex FP64):
  X1[z][kx][y] (2D: X1[kx][y]), X2[kx][ky][z], spectrum octant S[k][k][k].
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1501_04438_amd as gs

pytestmark = pytest.mark.gpu
TOL = 1e-13


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def fold(n):
    k = np.arange(2 * n)
    return np.minimum(k, 2 * n - k)


@pytest.mark.parametrize("n", [8, 12, 24, 64, 256])
def test_3d_passes(n):
    rng = np.random.default_rng(n)
    plan = gs.Plan("coulomb3d", n=n, L=5.0, slab_planes=-1)
    dev = "cuda:0"
    rho = rng.standard_normal((n, n, n))
    rt = torch.from_numpy(rho).to(dev)
    ut = torch.empty_like(rt)

    # P1: rho[z][y][x] -> X1[z][kx][y]
    plan.eval_pass(rt, ut, 1)
    got = plan.buffer(1)
    ref = np.fft.fft(rho, n=2 * n, axis=2)[:, :, : n + 1].transpose(0, 2, 1)
    assert rel(got, ref) < TOL, "P1"

    # P2: X1[z][kx][y] -> X2[kx][ky][z]
    x1 = crandn(rng, (n, n + 1, n))
    plan.buffer(1, x1)
    plan.eval_pass(rt, ut, 2)
    got = plan.buffer(2)
    ref = np.fft.fft(x1, n=2 * n, axis=2).transpose(1, 2, 0)
    assert rel(got, ref) < TOL, "P2"

    # P3: along z, forward (padded), times S[kx][|ky|][|kz|], inverse (cropped)
    S = plan.buffer(3)
    x2 = crandn(rng, (n + 1, 2 * n, n))
    plan.buffer(2, x2)
    plan.eval_pass(rt, ut, 3)
    got = plan.buffer(2)
    f = fold(n)
    Sf = S[:, f][:, :, f]                                   # [kx][ky][kz] over the padded ky, kz
    ref = (np.fft.ifft(np.fft.fft(x2, n=2 * n, axis=2) * Sf, axis=2) * 2 * n)[:, :, :n]
    assert rel(got, ref) < TOL, "P3"

    # P4: X2[kx][ky][z] -> X1[z][kx][y], y < n
    x3 = crandn(rng, (n + 1, 2 * n, n))
    plan.buffer(2, x3)
    plan.eval_pass(rt, ut, 4)
    got = plan.buffer(1)
    ref = (np.fft.ifft(x3, axis=1) * 2 * n)[:, :n, :].transpose(2, 0, 1)
    assert rel(got, ref) < TOL, "P4"

    # P5: X1[z][kx][y] (Hermitian half, DC and Nyquist real) -> u[z][y][x]
    x4 = crandn(rng, (n, n + 1, n))
    x4[:, 0, :] = x4[:, 0, :].real
    x4[:, n, :] = x4[:, n, :].real
    plan.buffer(1, x4)
    plan.eval_pass(rt, ut, 5)
    torch.cuda.synchronize()
    got = ut.cpu().numpy()
    ref = (np.fft.irfft(x4.transpose(0, 2, 1), n=2 * n, axis=2) * 2 * n)[:, :, :n]
    assert rel(got, ref) < TOL, "P5"


@pytest.mark.parametrize("n", [8, 48, 1024])
def test_2d_passes(n):
    rng = np.random.default_rng(n)
    plan = gs.Plan("coulomb2d", n=n, L=5.0)
    rho = rng.standard_normal((n, n))
    rt = torch.from_numpy(rho).to("cuda:0")
    ut = torch.empty_like(rt)
    plan.eval_pass(rt, ut, 1)
    ref = np.fft.fft(rho, n=2 * n, axis=1)[:, : n + 1].T
    assert rel(plan.buffer(1), ref) < TOL, "P1"
    S = plan.buffer(3)
    x = crandn(rng, (n + 1, n))
    # the pencils kx = 0 and kx = n are real, as P1 leaves them (the fused pass at n = 1024
    # transforms them together as one complex pencil)
    x[0] = x[0].real
    x[n] = x[n].real
    plan.buffer(1, x)
    plan.eval_pass(rt, ut, 3)
    ref = (np.fft.ifft(np.fft.fft(x, n=2 * n, axis=1) * S[:, fold(n)], axis=1) * 2 * n)[:, :n]
    assert rel(plan.buffer(1), ref) < TOL, "P3"
    x4 = crandn(rng, (n + 1, n))
    x4[0] = x4[0].real
    x4[n] = x4[n].real
    plan.buffer(1, x4)
    plan.eval_pass(rt, ut, 5)
    torch.cuda.synchronize()
    ref = (np.fft.irfft(x4.T, n=2 * n, axis=1) * 2 * n)[:, :n]
    assert rel(ut.cpu().numpy(), ref) < TOL, "P5"


@pytest.mark.parametrize("n,slabs", [(64, 0), (48, 5)])
def test_eval_events_same_bits_and_times(n, slabs):
    """gs_eval_events: the evaluation's steps back to back with an event after each; the
    output equals gs_eval's bit for bit, every interval is a positive time, NULL entries
    record nothing, and a wrong event count is refused."""
    import ctypes as C
    hip = C.CDLL("libamdhip64.so")
    hip.hipEventCreateWithFlags.argtypes = [C.POINTER(C.c_void_p), C.c_uint]
    hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
    hip.hipEventDestroy.argtypes = [C.c_void_p]
    plan = gs.Plan("coulomb3d", n=n, L=5.0, slab_planes=slabs)
    S = len(plan.steps())
    ev = []
    for _ in range(S + 1):
        e = C.c_void_p()
        assert hip.hipEventCreateWithFlags(C.byref(e), 0x20000000) == 0
        ev.append(e)
    rng = np.random.default_rng(n)
    rt = torch.from_numpy(rng.standard_normal((n, n, n))).to("cuda:0")
    ref = plan.eval(rt)
    ut = torch.empty_like(rt)
    plan.eval_events(rt, ut, ev)
    torch.cuda.synchronize()
    assert torch.equal(ut, ref)
    for a, b in zip(ev[:-1], ev[1:]):
        ms = C.c_float()
        assert hip.hipEventElapsedTime(C.byref(ms), a, b) == 0
        assert ms.value >= 0.0
    # NULL entries record nothing: events around one fused-pass launch only
    i = plan.steps().index(3)
    marks = [e if j in (i, i + 1) else None for j, e in enumerate(ev)]
    ut.zero_()
    plan.eval_events(rt, ut, marks)
    torch.cuda.synchronize()
    assert torch.equal(ut, ref)
    ms = C.c_float()
    assert hip.hipEventElapsedTime(C.byref(ms), ev[i], ev[i + 1]) == 0
    assert ms.value >= 0.0
    with pytest.raises(gs.GSError):
        plan.eval_events(rt, ut, ev[:-1])
    for e in ev:
        hip.hipEventDestroy(e)
