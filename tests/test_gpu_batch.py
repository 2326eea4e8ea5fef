"""Batched evaluation on the GPU: every schedule gives each problem bitwise the
result of its own evaluation, which the single-problem parity tests tie to the
oracle; small members are also checked against the oracle directly."""

import json
import os

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


# mixed kernels, dimensions and sizes, ragged tails (12, 24, 48, 96), every batch size
MIXED = [("coulomb3d", 32, 10.0), ("coulomb3d", 48, 10.0), ("coulomb3d", 24, 6.0), ("coulomb3d", 64, 10.0),
         ("coulomb3d", 12, 3.0), ("coulomb3d", 96, 8.0), ("coulomb3d", 128, 10.0), ("coulomb3d", 8, 2.0),
         ("coulomb3d", 16, 4.0), ("dipolar3d", 16, 4.0), ("dipolar3d", 24, 5.0), ("coulomb2d", 48, 7.0),
         ("poisson2d", 128, 7.0), ("coulomb2d", 8, 2.0),
         # the other kernel families and rectangular boxes share the batch path
         ("davey_stewartson2d", 24, 6.0), ("inverse_power", 16, 5.0), ("coulomb3d", 24, (3.0, 5.0, 8.0)),
         ("dipolar3d", 16, (4.0, 5.0, 6.0)), ("inverse_power", 48, (4.0, 4.0, 6.0))]


def member_kw(k):
    """Options of a member kernel, the same for the library and the oracle."""
    if k == "dipolar3d":
        return {"dipole": ((0.6, 0.8, 0.0), (0.0, 0.6, 0.8))}
    if k in ("poisson2d", "davey_stewartson2d"):
        return {"eps": 1e-13}
    if k == "inverse_power":
        return {"beta": 0.7}
    return {}


def make_plans(specs):
    return [gs.Plan(k, n=n, L=L, d=3 if k == "inverse_power" else None, **member_kw(k)) for k, n, L in specs]


@pytest.fixture(scope="module")
def mixed():
    plans = make_plans(MIXED)
    rng = np.random.default_rng(21)
    rhos = [cuda(rng.standard_normal(p.shape)) for p in plans]
    refs = [p.eval(r).clone() for p, r in zip(plans, rhos)]
    torch.cuda.synchronize()
    return plans, rhos, refs


@pytest.mark.parametrize("schedule,tpt", [("sequential", 1), ("phased", 1), ("phased", 2), ("sized", 1),
                                          ("sized", 3), ("queue", 1), ("queue", 3), ("concurrent", 1),
                                          ("concurrent", 3), ("streams", 1)])
@pytest.mark.parametrize("graph", [False, True])
def test_schedules_bitwise_equal_single(mixed, schedule, tpt, graph):
    plans, rhos, refs = mixed
    print(f"batch schedule={schedule} tiles_per_task={tpt} graph={graph}", flush=True)
    b = gs.Batch(plans, schedule=schedule, graph=graph, tiles_per_task=tpt)
    for rep in range(3):                                   # replays (graph) with eager work between
        outs = b.eval(rhos)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert torch.equal(o, r), (rep, MIXED[i])
        _ = (rhos[0] * 2.0).sum().item()
    info = b.info
    assert info["schedule"] == schedule and info["count"] == len(plans)
    assert info["wait_timeouts"] == 0
    if schedule not in ("sequential", "streams"):
        assert info["num_tasks"] == sum(info["tasks_per_pass"])
    if schedule == "queue":
        # one queue per die of the device, problems pinned to a die
        assert info["num_queues"] >= 1 and info["local_queues"] == (1 if info["num_queues"] >= 1 else 0)
    b.close()


def test_new_pointers_and_alias(mixed):
    """A second call with other tensors (descriptors re-uploaded, graph kept), then u aliasing rho."""
    plans, rhos, refs = mixed
    for schedule in ("queue", "phased", "sized", "concurrent", "streams"):
        b = gs.Batch(plans, schedule=schedule, graph=True)
        b.eval(rhos)
        copies = [r.clone() for r in rhos]
        outs = b.eval(copies, outs=copies)               # in place
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r)
        b.close()


def test_small_members_against_oracle(mixed):
    plans, rhos, _ = mixed
    outs = gs.Batch(plans, schedule="queue").eval(rhos)
    torch.cuda.synchronize()
    for (k, n, L), p, r, o in zip(MIXED, plans, rhos, outs):
        if n > 24:
            continue
        ref = oracle.evaluate(oracle.make_plan(k, p.d, n, L, **member_kw(k)), r.cpu().numpy())
        assert relmax(o.cpu().numpy(), ref) <= TOL, (k, n)


def test_one_shot_eval_batch(mixed):
    plans, rhos, refs = mixed
    outs = gs.eval_batch(plans, rhos)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)


def test_autotune_picks_a_schedule_and_caches_it(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("GS_AUTOTUNE_CACHE", str(path))
    probs = [workloads.materialise(p) for p in workloads.config4(6)]
    plans = [gs.Plan("coulomb3d", n=p.n, L=p.L) for p in probs]
    rhos = [cuda(p.rho) for p in probs]
    refs = [p.eval(r).clone() for p, r in zip(plans, rhos)]
    b = gs.Batch(plans, schedule="auto")
    outs = b.eval(rhos)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)
    info = b.info
    assert info["autotuned"] == 1 and info["candidates"] >= 2 and info["schedule"] != "auto"
    entries = json.loads(path.read_text())
    assert len(entries) == 1
    (key, e), = entries.items()
    assert e["schedule"] == gs.SCHEDULES[info["schedule"]] and e["ms"] > 0
    # a second batch of the same shapes takes the cached choice without timing
    b2 = gs.Batch(plans, schedule="auto")
    b2.eval(rhos)
    assert b2.info["candidates"] == 0 and b2.info["schedule"] == info["schedule"]


def test_batch_rejects_bad_input(mixed):
    plans, rhos, _ = mixed
    with pytest.raises(gs.GSError):
        gs.Batch([plans[0], plans[0]])
    big = gs.Plan("coulomb3d", n=256, L=10.0)
    with pytest.raises(gs.GSError):
        gs.Batch([plans[0], big], schedule="queue")
    with pytest.raises(gs.GSError):
        gs.Batch([plans[0], big], schedule="concurrent")
    # the automatic schedule falls back to the plans' own solves (in order or on concurrent
    # streams) for sizes beyond the batched kernels
    b = gs.Batch([plans[0], big], schedule="auto")
    r2 = cuda(np.random.default_rng(1).standard_normal((256,) * 3))
    outs = b.eval([rhos[0], r2])
    torch.cuda.synchronize()
    assert b.info["schedule"] in ("sequential", "streams")
    assert torch.equal(outs[1], big.eval(r2))


def test_config4_batch_of_64():
    """The batched workload: 64 mixtures on grids of 32..128 points per axis."""
    probs = [workloads.materialise(p) for p in workloads.config4(64)]
    plans = [gs.Plan("coulomb3d", n=p.n, L=p.L) for p in probs]
    rhos = [cuda(p.rho) for p in probs]
    outs = gs.Batch(plans, schedule="queue", graph=True).eval(rhos)
    torch.cuda.synchronize()
    for p, r, o in zip(plans, rhos, outs):
        assert torch.equal(o, p.eval(r))
    # the smallest member against the oracle
    i = min(range(64), key=lambda k: probs[k].n)
    ref = oracle.evaluate(oracle.make_plan("coulomb3d", 3, probs[i].n, probs[i].L), probs[i].rho)
    assert relmax(outs[i].cpu().numpy(), ref) <= TOL


def test_queue_schedule_small_grid_is_raised(mixed):
    """With per-die queues a grid below the co-resident block count would leave the
    queues of dies without blocks undrained: the library raises it, the results stay
    bitwise those of single evaluations and the error flag stays clear."""
    plans, rhos, refs = mixed
    b = gs.Batch(plans, schedule="queue", grid=3)
    outs = b.eval(rhos)
    torch.cuda.synchronize()
    info = b.info
    assert info["wait_timeouts"] == 0
    if info["local_queues"]:
        assert info["grid"] > 3
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)
    b.close()


def test_batch_follows_the_current_stream(mixed):
    """Batch.eval orders its work after the stream current at the call, not the one
    current at creation: inputs written on a side stream are read after that write."""
    plans, rhos, refs = mixed
    b = gs.Batch(plans, schedule="phased")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        copies = [torch.empty_like(r) for r in rhos]
        for c, r in zip(copies, rhos):
            c.copy_(r)
        outs = b.eval(copies)
    side.synchronize()
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)
    b.close()
