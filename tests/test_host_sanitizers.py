"""The library's host-side plan code (csrc/host_plan.cpp) built with g++ under the address
and undefined-behaviour sanitizers, run on small cubic and rectangular grids, and its
results compared with the oracle (tables, Taylor constants, the spectrum's first entry)."""

import math
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver_output(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("san") / "host_plan_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", os.path.join(HERE, "native", "host_plan_driver.cpp"),
           os.path.join(ROOT, "paper_1501_04438_amd", "csrc", "host_plan.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    out = {}
    for line in r.stdout.splitlines():
        name, rest = line.split(" ", 1)
        out[name] = {k: float(v) for k, v in re.findall(r"(\w+)=([-+0-9.eE]+)", rest)}
    return out


CASES = {
    "coulomb3d": ("coulomb3d", 3, 12, 4.0, 1e-14, None),
    "coulomb3d_rect": ("coulomb3d", 3, 12, (3.0, 4.0, 5.0), 1e-14, None),
    "poisson2d_rect": ("poisson2d", 2, 24, (6.0, 9.0), 1e-13, None),
    "ds2d": ("davey_stewartson2d", 2, 24, (6.0, 9.0), 1e-13, None),
    "power3d": ("inverse_power", 3, 12, (3.0, 4.0, 5.0), 1e-14, 0.7),
}


@pytest.mark.parametrize("name", list(CASES))
def test_sanitized_host_plan_matches_oracle(driver_output, name):
    kernel, d, n, L, eps, beta = CASES[name]
    got = driver_output[name]
    op = oracle.make_plan(kernel, d, n, L, eps=eps, beta=beta)
    assert abs(got["S"] - op.table.S) <= 1 and got["Q"] > 0
    dl = op.table.delta
    p = (d - beta) if beta else 2
    assert abs(got["A0"] - op.A0) <= 1e-10 * max(abs(op.A0), dl ** p)
    # the first spectrum entry: G at k = 0 plus A0, over M (zero for the d_xx symbol)
    ref0 = (op.G_oct.flat[0] + op.A0) / (2 * n) ** d
    if kernel == "davey_stewartson2d":
        assert got["spec0"] == 0.0
    else:
        assert abs(got["spec0"] - ref0) <= 1e-12 * abs(ref0)
    assert got["tw"] == 4 * n
