"""Writes oracle values at sampled grid points for the full-size workloads.

The oracle at 256^3 takes minutes and ~10 GB, too long to run inside a GPU
test; this script runs it once and stores, per workload, seeded sample indices,
the oracle's potential there and its max |u| over the whole grid.  It calls
only `oracle` and `workloads`.  Usage: python tests/golden/make_oracle_samples.py [name ...]
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402
import workloads   # noqa: E402

NSAMPLES = 4096


def _problem(name):
    if name == "c2_coulomb3d_256":
        return workloads.config2(256), {}
    if name == "c3_poisson2d_2048":
        return workloads.config3_2d("poisson2d", 2048), {"eps": 1e-13}
    if name == "c3_coulomb2d_2048":
        return workloads.config3_2d("coulomb2d", 2048), {}
    if name == "c3_dipolar3d_128":
        p = workloads.config3_dipolar(128)
        return p, {"dipole": (p.extra["n"], p.extra["m"])}
    raise KeyError(name)


NAMES = ["c2_coulomb3d_256", "c3_poisson2d_2048", "c3_coulomb2d_2048", "c3_dipolar3d_128"]


def make(name):
    p, kw = _problem(name)
    t = time.time()
    plan = oracle.make_plan(p.kernel, p.d, p.n, p.L, **kw)
    u = oracle.evaluate(plan, p.rho)
    rng = np.random.default_rng(7)
    idx = rng.integers(0, p.n, size=(NSAMPLES, p.d)).astype(np.int32)
    idx[0] = p.n // 2                                   # the centre
    vals = u[tuple(idx.T)]
    np.savez_compressed(os.path.join(HERE, f"oracle_{name}.npz"), idx=idx, u=vals,
                        umax=np.max(np.abs(u)), n=p.n, L=p.L, kernel=p.kernel,
                        energy=0.5 * plan.h ** p.d * float(np.sum(p.rho * u)))
    print(name, "done in %.1fs" % (time.time() - t), flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or NAMES):
        make(nm)
