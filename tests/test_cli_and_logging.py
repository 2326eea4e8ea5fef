"""Host-side behaviour that needs no GPU: the bench refuses more than one GPU with a
message, and GS_LOG_LEVEL makes the library report plan creation and errors on stderr."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_log_level_reports_plans_and_errors():
    code = ("import paper_1501_04438_amd as gs\n"
            "gs.Plan('coulomb3d', n=16, L=(3.0, 4.0, 5.0), host_only=True)\n"
            "try:\n    gs.Plan('coulomb3d', n=22, L=4.0, host_only=True)\nexcept gs.GSError:\n    pass\n")
    env = dict(os.environ, GS_LOG_LEVEL="2", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, env=env, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    assert "[gs] host-only plan kernel=0 d=3 n=(16, 16, 16) L=(3, 4, 5)" in r.stderr
    assert "[gs] error 2: no kernels compiled for transforms of n = 22" in r.stderr
    env["GS_LOG_LEVEL"] = "0"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, env=env, cwd=ROOT)
    assert "[gs]" not in r.stderr
