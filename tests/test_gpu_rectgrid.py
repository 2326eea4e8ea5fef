"""Grids whose axes have their own n (Section 2.5: the box prod_j [-L_j, L_j] with n_j
points on axis j; a box with unequal sides and one step h needs unequal n_j).

Each pass runs at the length of the axis it transforms (x passes at n_x, y passes at
n_y, the fused pass at n_z in 3D and n_y in 2D) with the other extents at run time.
HIP path through the C ABI against the oracle, element by element, max-norm
relative error <= 1e-12; ragged tiles (12, 24, 48, 96 on any axis), the 256 and 2048
lengths on one axis, every kernel family, slabs, energy, mixture gradients, the
adjoint and the allocation-free entry point."""

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_1501_04438_amd as gs
import workloads
from oracle import closed_forms as cf
from paper_1501_04438_amd._lib import lib

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
        return {"beta": 1.3}
    return {}


CASES = [("coulomb3d", 3, (12, 24, 16), (3.0, 6.0, 4.0)),
         ("coulomb3d", 3, (64, 96, 128), (4.0, 6.0, 8.0)),
         ("coulomb3d", 3, (96, 48, 64), (6.0, 3.0, 4.0)),
         ("coulomb3d", 3, (32, 16, 256), (2.0, 1.0, 16.0)),
         ("coulomb3d", 3, (8, 192, 24), (1.0, 24.0, 3.0)),
         ("dipolar3d", 3, (24, 16, 48), (3.0, 2.0, 6.0)),
         ("inverse_power", 3, (16, 32, 12), (4.0, 8.0, 3.0)),
         ("poisson2d", 2, (96, 192), (6.0, 12.0)),
         ("coulomb2d", 2, (192, 64), (12.0, 4.0)),
         ("coulomb2d", 2, (256, 2048), (2.0, 16.0)),
         # fused axis of 1024 points: its zero and Nyquist pencils (kx = 0, 96) ride together
         ("poisson2d", 2, (1024, 96), (12.0, 1.125)),
         ("davey_stewartson2d", 2, (32, 64), (4.0, 7.0)),
         ("inverse_power", 2, (48, 12), (8.0, 2.0))]


@pytest.mark.parametrize("kernel,d,n,L", CASES)
def test_random_input_against_oracle(kernel, d, n, L):
    print(f"rectangular grid: {kernel} n={n} L={L}", flush=True)
    kw = kw_of(kernel)
    rng = np.random.default_rng(sum(n))
    rho = rng.standard_normal(n)
    plan = gs.Plan(kernel, n=n, L=L, d=d, **kw)
    assert plan.info["n_axes"] == tuple(n)
    u = plan.eval(cuda(rho))
    torch.cuda.synchronize()
    ref = oracle.evaluate(oracle.make_plan(kernel, d, n, L, **kw), rho)
    assert relmax(u.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("kernel,n,L,sigma", [("coulomb3d", (64, 96, 128), (4.0, 6.0, 8.0), 0.6),
                                              ("poisson2d", (96, 192), (6.0, 12.0), 0.8)])
def test_gaussian_closed_form_equal_steps(kernel, n, L, sigma):
    """The same step h = 1/8 on unequal sides: the closed-form potential of a resolved
    Gaussian to 1e-13 of its maximum."""
    d = len(n)
    rho = workloads.gaussian(n, L, d, sigma=sigma)
    plan = gs.Plan(kernel, n=n, L=L, **kw_of(kernel))
    u = plan.eval(cuda(rho)).cpu().numpy()
    X = np.broadcast_arrays(*workloads.mesh(n, L, d))
    r = np.sqrt(sum(x * x for x in X))
    ex = cf.coulomb3d_gaussian(r, sigma) if kernel == "coulomb3d" else cf.poisson2d_gaussian(r, sigma)
    assert relmax(u, ex) <= 1e-13


def test_device_assembly_equals_host():
    for kernel, n, L in [("coulomb3d", (24, 12, 48), (3.0, 1.5, 6.0)), ("poisson2d", (64, 128), (4.0, 8.0))]:
        kw = kw_of(kernel)
        dev = gs.Plan(kernel, n=n, L=L, **kw).spectrum()
        host = gs.Plan(kernel, n=n, L=L, host_only=True, **kw).spectrum()
        assert dev.shape == tuple(m + 1 for m in reversed(n))
        assert np.max(np.abs(dev - host)) <= 1e-14 * np.max(np.abs(host))


def test_slabs_adjoint_energy_static():
    """kx slabs (same bits), the adjoint against the oracle's transposed steps and the dot
    test, the energy formed in the last pass, and gs_eval_static, on one rectangular grid."""
    n, L = (24, 48, 12), (3.0, 6.0, 1.5)
    rng = np.random.default_rng(5)
    a, v = rng.standard_normal(n), rng.standard_normal(n)
    plan = gs.Plan("coulomb3d", n=n, L=L)
    ua = plan.eval(cuda(a))
    for sp in (1, 4, 7):
        assert torch.equal(gs.Plan("coulomb3d", n=n, L=L, slab_planes=sp).eval(cuda(a)), ua)
    atv = plan.eval_backward(cuda(v))
    torch.cuda.synchronize()
    ref = oracle.adjoint(oracle.make_plan("coulomb3d", 3, n, L), v)
    assert relmax(atv.cpu().numpy(), ref) <= TOL
    lhs, rhs = float((ua * cuda(v)).sum()), float((cuda(a) * atv).sum())
    assert abs(lhs - rhs) <= 1e-14 * float(ua.norm() * atv.norm())
    u2, E = plan.eval_energy(cuda(a))
    assert torch.equal(u2, ua)
    Eo = oracle.energy(oracle.make_plan("coulomb3d", 3, n, L), a)
    prod = 0.5 * plan.cell * (cuda(a) * ua)
    assert abs(float(E) - Eo) <= 1e-13 * float(prod.abs().sum())
    bare = gs.Plan("coulomb3d", n=n, L=L, workspace=False)
    x = cuda(a)
    u3 = torch.empty_like(x)
    bare._stream()
    assert lib().gs_eval_static(bare._h, C.c_void_p(x.data_ptr()), C.c_void_p(u3.data_ptr())) == 0
    torch.cuda.synchronize()
    assert torch.equal(u3, ua)


@pytest.mark.parametrize("kernel,d,n,L,K", [("coulomb3d", 3, (32, 48, 24), (8.0, 12.0, 6.0), 6),
                                            ("poisson2d", 2, (96, 48), (12.0, 6.0), 9)])
def test_mixture_path_rectangular_grid(kernel, d, n, L, K):
    kw = kw_of(kernel)
    plan = gs.Plan(kernel, n=n, L=L, **kw)
    rng = np.random.default_rng(70 + K)
    t = lambda x: torch.tensor(x, dtype=torch.float64, device="cuda:0", requires_grad=True)
    a, mu, s = t(rng.uniform(-1, 1, K)), t(rng.uniform(-2, 2, (K, d))), t(rng.uniform(0.5, 1.5, K))
    rho = plan.mixture_density(a, mu, s)
    ref = gs.mixture_density(a.detach(), mu.detach(), s.detach(), n, L)
    assert float((rho - ref).abs().max()) <= 1e-15 * float(ref.abs().max())
    E = gs.mixture_energy(a, mu, s, plan)
    g = torch.autograd.grad(E, (a, mu, s))
    Eo, ga, gmu, gsig = oracle.energy_gradient_params(oracle.make_plan(kernel, d, n, L, **kw),
                                                      a.detach().cpu().numpy(), mu.detach().cpu().numpy(),
                                                      s.detach().cpu().numpy())
    got = np.concatenate([x.cpu().numpy().ravel() for x in g])
    go = np.concatenate([ga, gmu.ravel(), gsig])
    assert abs(float(E) - Eo) <= 1e-12 * abs(Eo)
    assert np.max(np.abs(got - go)) <= 1e-12 * np.max(np.abs(go))


def test_batch_takes_rectangular_grids_sequentially():
    """The batched kernels hold cubic grids only: an explicit batched schedule refuses a
    rectangular grid, the automatic one evaluates it by its own passes (same bits)."""
    rect = gs.Plan("coulomb3d", n=(16, 24, 32), L=(2.0, 3.0, 4.0))
    cube = gs.Plan("coulomb3d", n=32, L=4.0)
    with pytest.raises(gs.GSError):
        gs.Batch([rect, cube], schedule="queue")
    rng = np.random.default_rng(3)
    r1, r2 = cuda(rng.standard_normal(rect.shape)), cuda(rng.standard_normal(cube.shape))
    b = gs.Batch([rect, cube], schedule="auto")
    outs = b.eval([r1, r2])
    torch.cuda.synchronize()
    assert b.info["schedule"] in ("sequential", "streams")
    assert torch.equal(outs[0], rect.eval(r1)) and torch.equal(outs[1], cube.eval(r2))


def test_packed_pencils_energy_rectangular():
    """The 2D fused pass of 1024 points on a grid with 96 columns: the energy formed in the
    pass (the packed pencil's two spectra summed apart) against the sum in space, and the
    potential on the same bits as gs_eval."""
    n, L = (1024, 96), (12.0, 1.125)
    rng = np.random.default_rng(96)
    rho = cuda(rng.standard_normal(n))
    plan = gs.Plan("coulomb2d", n=n, L=L)
    u0 = plan.eval(rho)
    u, e = plan.eval_energy(rho)
    torch.cuda.synchronize()
    assert torch.equal(u, u0)
    cell = (2 * L[0] / n[0]) * (2 * L[1] / n[1])
    e_space = 0.5 * cell * float((rho * u).sum())
    assert abs(float(e) - e_space) <= 1e-13 * 0.5 * cell * float((rho * u).abs().sum())
