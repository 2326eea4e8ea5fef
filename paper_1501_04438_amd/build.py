"""Build of the HIP library libgs.so for gfx950 (in-tree, next to this file).

Objects: one evaluation-pass object per supported transform length (the
size list lives in csrc/sizes.hpp), the size dispatch and matrix-core
assembly, the host plan code and the C ABI.  Run `python -m
paper_1501_04438_amd.build` or call build().
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libgs.so")

ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++20", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sizes() -> list[int]:
    txt = open(os.path.join(CSRC, "sizes.hpp")).read()
    m = re.search(r"#define GS_SIZE_LIST\(X\)(.*)", txt)
    return [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return cmd[-1]


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = []
    for n in sizes():
        units.append([cc, *FLAGS, f"-DGS_N={n}", "-c", os.path.join(CSRC, "eval_instance.hip"),
                      "-o", os.path.join(BUILD, f"eval_{n}.o")])
    # The spectrum assembly (device_dispatch.hip holds the only matrix-core kernel) keeps its
    # MFMA accumulators in VGPRs: with the default accumulator-register form the compiler
    # copied all 72 accumulator dwords between VGPRs and AGPRs in every K step (144 moves per
    # 9 MFMAs); the VGPR form has none: 0.304 -> 0.245 ms at 256^3 (27.8 -> 34.5 TFLOP/s).
    # The mixture gradient's contraction (mixture.hip) is built the same way: 132 VGPRs and no
    # accumulator copies instead of 164 registers and 64 copies per tile.
    extra = {"device_dispatch.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
             "mixture.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}
    for src in ("device_dispatch.hip", "batch.hip", "host_plan.cpp", "gs_api.cpp", "batch_api.cpp",
                "autotune.cpp", "static_eval.hip", "mixture.hip"):
        units.append([cc, *FLAGS, *extra.get(src, []), "-c", os.path.join(CSRC, src),
                      "-o", os.path.join(BUILD, os.path.splitext(src)[0] + ".o")])
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_run, units))
    tmp = LIB + ".tmp"
    _run([cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
