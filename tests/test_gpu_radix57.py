"""Transform lengths with factors 5 and 7 (radix-5 and radix-7 stages: n = 5 * 2^a, 7 * 2^a).

HIP path through the C ABI against the oracle element by element (max-norm relative error
<= 1e-12) on cubes, squares and rectangular grids of these lengths, every kernel family;
3D 320^3 and 640^3 against the closed-form potential of a resolved Gaussian; tile variants,
slabs and the automatic batch give the same bits."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_1501_04438_amd as gs
import workloads
from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def kw_of(kernel):
    if kernel == "dipolar3d":
        return {"dipole": ((0.3, -0.5, 0.8), (0.9, 0.1, -0.2))}
    if kernel in ("poisson2d", "davey_stewartson2d"):
        return {"eps": 1e-13}
    if kernel == "inverse_power":
        return {"beta": 0.7}
    return {}


CASES = [("coulomb3d", 3, 20, 4.0), ("coulomb3d", 3, 28, 4.0), ("coulomb3d", 3, 40, 6.0),
         ("coulomb3d", 3, 56, 6.0), ("coulomb3d", 3, 80, 8.0), ("coulomb3d", 3, 112, 8.0),
         ("coulomb3d", 3, 160, 10.0), ("coulomb3d", 3, 224, 10.0),
         ("coulomb3d", 3, (20, 56, 40), (2.0, 5.6, 4.0)), ("coulomb3d", 3, (160, 28, 80), (16.0, 2.8, 8.0)),
         ("dipolar3d", 3, 40, 5.0), ("inverse_power", 3, 28, 3.0),
         ("poisson2d", 2, 320, 12.0), ("poisson2d", 2, 640, 12.0), ("coulomb2d", 2, 224, 9.0),
         ("coulomb2d", 2, (640, 112), (16.0, 2.8)), ("davey_stewartson2d", 2, 80, 6.0),
         ("inverse_power", 2, 160, 6.0)]


@pytest.mark.parametrize("kernel,d,n,L", CASES)
def test_random_input_against_oracle(kernel, d, n, L):
    print(f"radix 5/7 lengths: {kernel} n={n} L={L}", flush=True)
    kw = kw_of(kernel)
    plan = gs.Plan(kernel, n=n, L=L, d=d, **kw)
    rng = np.random.default_rng(500 + sum(np.atleast_1d(n)))
    rho = rng.standard_normal(plan.shape)
    u = plan.eval(cuda(rho))
    torch.cuda.synchronize()
    ref = oracle.evaluate(oracle.make_plan(kernel, d, n, L, **kw), rho)
    assert relmax(u.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("n,L", [(320, 16.0), (640, 16.0)])
def test_large_cubes_against_closed_form(n, L):
    """320^3 and 640^3 (h = 1/10, 1/20): a resolved Gaussian's potential to 1e-13 of its
    maximum, on a sampled set of points and the maximum over the whole grid."""
    print(f"radix 5 cube: n={n}", flush=True)
    plan = gs.Plan("coulomb3d", n=n, L=L)
    x = cuda(workloads.gaussian(n, L, 3, sigma=1.0))
    u = plan.eval(x)
    torch.cuda.synchronize()
    rng = np.random.default_rng(n)
    idx = rng.integers(0, n, size=(4000, 3))
    idx[:8] = [[n // 2, n // 2, n // 2], [0, 0, 0], [n - 1, n - 1, n - 1], [n // 2, 0, n - 1],
               [0, n // 2, n // 2], [n // 3, n // 4, n // 5], [n - 1, 0, 0], [1, 2, 3]]
    h = 2 * L / n
    got = u[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    pts = -L + h * idx.astype(np.float64)
    r = np.sqrt(np.sum(pts * pts, axis=1))
    ex = cf.coulomb3d_gaussian(r, 1.0)
    umax = float(cf.coulomb3d_gaussian(np.array([0.0]), 1.0)[0])
    assert np.max(np.abs(got - ex)) <= 1e-13 * umax
    assert abs(float(u.max()) - umax) <= 1e-13 * umax


def test_tile_variants_slabs_and_batch_same_bits():
    rng = np.random.default_rng(7)
    x = cuda(rng.standard_normal((160, 160, 160)))
    base = gs.Plan("coulomb3d", n=160, L=8.0)
    u0 = base.eval(x)
    for tv in (1, 1 << 2, 2 << 2, 1 << 4, 2 << 4, 1 << 6):
        assert torch.equal(gs.Plan("coulomb3d", n=160, L=8.0, tile_variants=tv).eval(x), u0), tv
    assert torch.equal(gs.Plan("coulomb3d", n=160, L=8.0, slab_planes=9).eval(x), u0)
    small = gs.Plan("coulomb3d", n=40, L=4.0)
    y = cuda(rng.standard_normal((40, 40, 40)))
    b = gs.Batch([base, small], schedule="auto")
    outs = b.eval([x, y])
    torch.cuda.synchronize()
    assert torch.equal(outs[0], u0) and torch.equal(outs[1], small.eval(y))


def test_adjoint_and_energy():
    n, L = (40, 28, 20), (4.0, 2.8, 2.0)
    plan = gs.Plan("coulomb3d", n=n, L=L)
    rng = np.random.default_rng(11)
    a, v = rng.standard_normal(n), rng.standard_normal(n)
    ua, atv = plan.eval(cuda(a)), plan.eval_backward(cuda(v))
    torch.cuda.synchronize()
    op = oracle.make_plan("coulomb3d", 3, n, L)
    assert relmax(atv.cpu().numpy(), oracle.adjoint(op, v)) <= TOL
    u2, E = plan.eval_energy(cuda(a))
    assert torch.equal(u2, ua)
    assert abs(float(E) - oracle.energy(op, a)) <= 1e-13 * float((0.5 * plan.cell * (cuda(a) * ua)).abs().sum())
