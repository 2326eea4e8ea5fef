"""Full-size parity: the HIP path against the oracle at every grid point.

The workloads at their full sizes, in the launch configuration the benchmark
times (default plans: the persistent fused pass at 256^3, one block per pencil
group elsewhere), compared element by element with `oracle.evaluate` computed
inside the test (a few seconds to tens of seconds on the host cores, about
10 GB at 256^3).  Bar: max-norm relative error (eq. (error_infty)) <= 1e-12.

  * the headline workload: 3D Coulomb mixture at 256^3 (the only size that runs
    the persistent fused pass);
  * the 2D mixtures at 2048^2 for the Poisson and 2D Coulomb kernels;
  * a rough (random) 3D Coulomb input at 192^3 (a 12-value transform plan);
  * the dipolar kernel at 256^3 (the persistent dipolar fused pass) with the
    printed orientations of the dipolar example and with seeded ones, and at 128^3;
  * every member of the 64-problem batch through the one-launch queue schedule.
"""

import gc

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_1501_04438_amd as gs
import workloads

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


def gpu_eval(plan, rho):
    u = plan.eval(cuda(rho))
    torch.cuda.synchronize()
    out = u.cpu().numpy()
    del u
    return out


def _free():
    gc.collect()
    torch.cuda.empty_cache()


def _compare(p, kw, label):
    print(f"full-size parity: {label} ({p.kernel}, n={p.n}, L={p.L})", flush=True)
    plan = gs.Plan(p.kernel, n=p.n, L=p.L, **kw)
    u = gpu_eval(plan, p.rho)
    del plan
    _free()
    ref = oracle.evaluate(oracle.make_plan(p.kernel, p.d, p.n, p.L, **kw), p.rho)
    err = relmax(u, ref)
    print(f"  max-norm relative error {err:.3e}", flush=True)
    return u, ref, err


def test_headline_coulomb3d_256_every_point():
    p = workloads.config2(256)
    u, ref, err = _compare(p, {}, "config 2 headline mixture")
    assert err <= TOL, err
    # the energy 1/2 h^3 sum rho u on the scale of sum |rho u|
    h3 = (2.0 * p.L / p.n) ** 3
    scale = 0.5 * h3 * float(np.sum(np.abs(p.rho * ref)))
    assert abs(0.5 * h3 * float(np.sum(p.rho * u)) - 0.5 * h3 * float(np.sum(p.rho * ref))) <= 1e-13 * scale
    del u, ref
    _free()


@pytest.mark.parametrize("kernel", ["poisson2d", "coulomb2d"])
def test_2d_mixture_2048_every_point(kernel):
    p = workloads.config3_2d(kernel, 2048)
    kw = {"eps": 1e-13} if kernel == "poisson2d" else {}
    _, _, err = _compare(p, kw, "config 3 mixture")
    assert err <= TOL, err
    _free()


def test_coulomb3d_random_192_every_point():
    n = 192
    rho = np.random.default_rng(192).standard_normal((n, n, n))
    p = workloads.Problem("coulomb3d", 3, n, 9.0, rho)
    _, _, err = _compare(p, {}, "random input")
    assert err <= TOL, err
    _free()


@pytest.mark.parametrize("n,paper", [(256, True), (256, False), (128, False)])
def test_dipolar_every_point(n, paper):
    p = workloads.config3_dipolar(n, paper_vectors=paper)
    kw = {"dipole": (p.extra["n"], p.extra["m"])}
    _, _, err = _compare(p, kw, "dipolar, " + ("printed vectors" if paper else "seeded vectors"))
    assert err <= TOL, err
    _free()


def test_batch_of_64_every_member_every_point():
    """The 64-problem batch through the one-launch queue schedule (graph replay): every
    member against the oracle at every grid point."""
    probs = [workloads.materialise(p) for p in workloads.config4(64)]
    print(f"batch of 64: sizes {sorted(set(p.n for p in probs))}", flush=True)
    plans = [gs.Plan("coulomb3d", n=p.n, L=p.L) for p in probs]
    rhos = [cuda(p.rho) for p in probs]
    b = gs.Batch(plans, schedule="queue", graph=True)
    outs = b.eval(rhos)
    torch.cuda.synchronize()
    assert b.info["wait_timeouts"] == 0
    got = [o.cpu().numpy() for o in outs]
    b.close()
    del outs, rhos, plans
    _free()
    oplans = {}
    worst = 0.0
    for i, p in enumerate(probs):
        if p.n not in oplans:
            oplans[p.n] = oracle.make_plan("coulomb3d", 3, p.n, p.L)
        err = relmax(got[i], oracle.evaluate(oplans[p.n], p.rho))
        worst = max(worst, err)
        assert err <= TOL, (i, p.n, err)
    print(f"  worst member error {worst:.3e}", flush=True)
