#!/usr/bin/env python3
"""Benchmark of the Gaussian-sum potential evaluation on one MI355X.

Metric: Mpts/s per potential evaluation, 3D Coulomb, n = 256 per axis, FP64,
accuracy <= 1e-12 against the oracle.  Workload: the triaxial Gaussian
exp(-(x^2 + 4y^2 + 16z^2)) plus an 8-component seeded Gaussian mixture on
[-10, 10]^3 (workloads.config2), density resident in HBM, plan (tables,
factors, spectrum assembly) built before the timed region, as the paper times
evaluations only.  One step = one evaluation (all five passes).

Each step of the timed loop is one library call that launches the five passes
back to back with HIP timing events (no system-scope fence) recorded between
them on the launching stream, which gives every pass's device time; the
dominant pass is reported against the HBM roofline with its algorithmic bytes.
Also reported: the oracle on a bounded sample of the same workload on the host
cores (cpu_baseline), the batched (64 uneven problems) and adjoint figures.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix
PASS_NAMES = {1: "k_x_r2c", 2: "k_y_fwd", 3: "k_fused", 4: "k_y_inv", 5: "k_x_c2r"}
KERNEL_SOURCES = ["paper_1501_04438_amd/csrc/passes.hpp", "paper_1501_04438_amd/csrc/fft_core.hpp",
                  "paper_1501_04438_amd/csrc/eval_instance.hip"]


def pass_bytes(n: int) -> dict:
    """Algorithmic HBM bytes per launch of each 3D pass (each input read once,
    each output written once, spectrum octant read once)."""
    n1 = n + 1
    x1 = 16 * n1 * n * n          # [z][kx][y] complex
    x2 = 32 * n1 * n * n          # [kx][ky][z] complex
    real = 8 * n ** 3
    return {1: real + x1, 2: x1 + x2, 3: 2 * x2 + 8 * n1 ** 3, 4: x2 + x1, 5: x1 + real}


def source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_coulomb3d_256.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != source_hash():
        return None
    return t.get("kernels", {}).get(kernel, {}).get("bytes_per_launch")


# The three profiled runs behind profiles/ (from the repository root, TMPDIR=/tmp, output
# folders under {out}); each counter pass is its own run, bounded by a kill timeout.
PROFILE_STEPS = (
    "timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d {out}/pmc_fetch -o run --output-format csv "
    "-- python3 bench.py --steps 5 --warmup 1 --no-extras --no-cpu-baseline",
    "timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d {out}/pmc_write -o run --output-format csv "
    "-- python3 bench.py --steps 5 --warmup 1 --no-extras --no-cpu-baseline",
    "timeout -s KILL 180 rocprofv3 --kernel-trace --stats -d {out}/ktrace -o run --output-format csv "
    "-- python3 bench.py --steps 20 --warmup 3 --no-extras --no-cpu-baseline")


def profile_steps(out: str) -> list:
    return [c.format(out=out) for c in PROFILE_STEPS]


def _csv_rows(directory: str, suffix: str):
    import csv
    import glob
    paths = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not paths:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    with open(paths[0]) as f:
        return list(csv.DictReader(f))


def summarize_profiles(fetch_dir: str, write_dir: str, trace_dir: str, n: int = 256) -> int:
    """HBM traffic per launch of each pass from two rocprofv3 counter runs (FETCH_SIZE,
    WRITE_SIZE in KiB per dispatch) and the kernel-duration table from a kernel-trace
    run, all of `python3 bench.py --no-extras --no-cpu-baseline` (PROFILE_STEPS).  Each
    counter is scaled by what it reads for the bench's 2 GiB device-to-device copies
    (2 GiB read and 2 GiB written by definition)."""
    import statistics
    copy_bytes = 2048 * 2 ** 20
    names = list(PASS_NAMES.values())

    def per_kernel(rows, counter):
        out = {k: [] for k in names}
        copies = []
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0          # KiB -> bytes
            kn = r["Kernel_Name"]
            for k in names:
                if k in kn:
                    out[k].append(v)
            if "copyBuffer" in kn and v > 0.25 * 2 ** 30:
                copies.append(v)
        return out, copies

    fetch, fcopies = per_kernel(_csv_rows(fetch_dir, "counter_collection.csv"), "FETCH_SIZE")
    write, wcopies = per_kernel(_csv_rows(write_dir, "counter_collection.csv"), "WRITE_SIZE")
    fscale = copy_bytes / statistics.median(fcopies)
    wscale = copy_bytes / statistics.median(wcopies)
    nb = pass_bytes(n)
    kern = {}
    for p, k in PASS_NAMES.items():
        if not fetch[k] or not write[k]:
            continue
        fb = statistics.mean(fetch[k]) * fscale
        wb = statistics.mean(write[k]) * wscale
        kern[k] = {"fetch_bytes": round(fb), "write_bytes": round(wb), "bytes_per_launch": round(fb + wb),
                   "alg_bytes": nb[p], "ratio_to_alg": round((fb + wb) / nb[p], 3)}
    out = os.path.dirname(os.path.normpath(fetch_dir)) or "."
    steps = profile_steps(out)
    traffic = {"source_hash": source_hash(), "n": n, "command": " && ".join(steps),
               "fetch_scale": round(fscale, 4), "write_scale": round(wscale, 4),
               "calibration": "median FETCH_SIZE / WRITE_SIZE of the bench's 2 GiB device-to-device copies",
               "kernels": kern}
    with open(os.path.join(ROOT, "profiles", f"traffic_coulomb3d_{n}.json"), "w") as f:
        json.dump(traffic, f, indent=1)

    rows = _csv_rows(trace_dir, "kernel_stats.csv")
    lines = [f"# Kernel durations: 3D Coulomb {n}^3 evaluation", "",
             "Command (from the repository root on an MI355X, TMPDIR=/tmp):", "", "    " + steps[2], "",
             f"Source: {trace_dir}/.../run_kernel_stats.csv.  k_assemble is the plan-time spectrum assembly;",
             "__amd_rocclr_copyBuffer are the density upload and the bench's copy-bandwidth probe.", "",
             "| kernel | calls | average ns | min ns | max ns | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r.get("Name", r.get("Kernel_Name", "?"))
        short = name.split("(")[0].replace("void ", "").replace("gsk::", "")
        lines.append(f"| {short[:60]} | {r.get('Calls')} | {float(r.get('AverageNs', 0)):.0f} | "
                     f"{float(r.get('MinNs', 0)):.0f} | {float(r.get('MaxNs', 0)):.0f} | "
                     f"{float(r.get('Percentage', 0)):.1f} |")
    lines += loop_table(trace_dir, steps[2])
    lines += ["", "HBM traffic per launch (FETCH_SIZE x %.3f + WRITE_SIZE x %.3f, bytes):" % (fscale, wscale), "",
              "| kernel | fetch | write | total | algorithmic | ratio |", "|---|---|---|---|---|---|"]
    for k, v in kern.items():
        lines.append(f"| {k} | {v['fetch_bytes']} | {v['write_bytes']} | {v['bytes_per_launch']} | "
                     f"{v['alg_bytes']} | {v['ratio_to_alg']} |")
    lines += ["", "Counter commands:", ""] + ["    " + c for c in steps[:2]]
    with open(os.path.join(ROOT, "profiles", f"eval_coulomb3d_{n}_kernel_stats.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(traffic, indent=1))
    return 0


def loop_table(trace_dir: str, command: str) -> list:
    """Mean duration of each pass kernel in each loop of one bench run, from the kernel
    trace (launches in start order; each evaluation launches each pass once): warmup, the
    loop with an event after every pass, the loops with events around one other pass, the
    timed loop (events around the dominant kernel only) and the loop without events."""
    import re
    import statistics
    W = int(re.search(r"--warmup (\d+)", command).group(1))
    K = int(re.search(r"--steps (\d+)", command).group(1))
    rows = sorted(_csv_rows(trace_dir, "kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"]))
    seq = {k: [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows if k in r["Kernel_Name"]]
           for k in PASS_NAMES.values()}
    loops = [("warmup", 0, W), ("event after every pass", W, W + K),
             ("events around one other pass", W + K, W + 5 * K),
             ("timed: events around the dominant kernel", W + 5 * K, W + 6 * K),
             ("no events", W + 6 * K, W + 7 * K)]
    out = ["", "Mean duration per loop of the run (us, from run_kernel_trace.csv):", "",
           "| loop | evaluations | " + " | ".join(PASS_NAMES.values()) + " |", "|---|---|" + "---|" * len(PASS_NAMES)]
    for name, a, b in loops:
        cells = [f"{statistics.mean(v[a:b]):.1f}" if len(v) >= b else "-" for v in seq.values()]
        out.append(f"| {name} | {b - a} | " + " | ".join(cells) + " |")
    return out


class HipEvents:
    """Timing events of the HIP runtime (ctypes), created with hipEventDisableSystemFence."""

    FLAGS = 0x20000000          # hipEventDisableSystemFence

    def __init__(self):
        import ctypes
        self.C = ctypes
        self.lib = ctypes.CDLL("libamdhip64.so")
        self.lib.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        self.lib.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def _check(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed ({rc})")

    def create(self):
        e = self.C.c_void_p()
        self._check(self.lib.hipEventCreateWithFlags(self.C.byref(e), self.FLAGS), "hipEventCreateWithFlags")
        return e

    def record(self, e, stream):
        self._check(self.lib.hipEventRecord(e, self.C.c_void_p(stream)), "hipEventRecord")

    def elapsed(self, a, b) -> float:
        ms = self.C.c_float()
        self._check(self.lib.hipEventElapsedTime(self.C.byref(ms), a, b), "hipEventElapsedTime")
        return float(ms.value)

    def destroy(self, events):
        for e in events:
            self.lib.hipEventDestroy(e)


def cpu_baseline(n_sample: int, min_seconds: float = 10.0) -> dict:
    """The oracle, as it stands, on the same workload: whole evaluations repeated
    until at least min_seconds of host time (plan construction excluded)."""
    import oracle
    import workloads
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:
        threads = os.cpu_count() or 1
    p = workloads.config2(n_sample)
    plan = oracle.make_plan("coulomb3d", 3, n_sample, p.L, eps=1e-14)
    evals, dt = 0, 0.0
    u_ref = None
    while dt < min_seconds:
        t0 = time.perf_counter()
        u_ref = oracle.evaluate(plan, p.rho)
        dt += time.perf_counter() - t0
        evals += 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    out = {"value": evals * n_sample ** 3 / dt / 1e6, "unit": "Mpts/s", "cores": int(threads), "kind": "oracle",
           "cpu_model": model,
           "sample": f"{evals} evaluation(s) of the same workload at {n_sample}^3 (plan excluded), {dt:.1f} s"}
    out["cpu_fft_reference"] = cpu_fft_reference(oracle, plan, p.rho, u_ref, int(threads))
    return out


def cpu_fft_reference(oracle, plan, rho, u_ref, workers: int) -> dict:
    """A fairer CPU speed comparison than the oracle (not the oracle): the same folded spectrum
    applied with scipy.fft on the zero-padded grid, u = crop(IFFT(S . FFT(pad rho))), on all
    host cores; one evaluation, its agreement with the oracle's output reported."""
    import numpy as np
    import scipy.fft as sf
    n = rho.shape[0]
    S = oracle.full_spectrum(plan) + plan.A0 - plan.c2 * oracle.laplacian_symbol(plan)
    rp = np.zeros((2 * n,) * 3)
    t0 = time.perf_counter()
    rp[:n, :n, :n] = rho
    X = sf.fftn(rp, workers=workers)
    X *= S
    u = sf.ifftn(X, workers=workers).real[:n, :n, :n]
    dt = time.perf_counter() - t0
    err = float(np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)))
    return {"value": n ** 3 / dt / 1e6, "unit": "Mpts/s", "cores": workers, "kind": "scipy.fft, folded spectrum",
            "sample": f"one evaluation at {n}^3, {dt:.2f} s", "max_rel_diff_vs_oracle": err}


def dgemm_tflops(torch, m: int = 8192, reps: int = 5) -> float:
    """FP64 matrix product of two m x m matrices (the vendor BLAS): the measured FP64 matrix
    peak, reported next to the datasheet's for the spectrum assembly."""
    a = torch.rand((m, m), dtype=torch.float64, device="cuda:0")
    b = torch.rand((m, m), dtype=torch.float64, device="cuda:0")
    c = a @ b
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        c = a @ b
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b, c
    return 2.0 * m ** 3 / (ms * 1e-3) / 1e12


def copy_bandwidth(torch, mib: int = 2048, reps: int = 20) -> float:
    """Device-to-device copy of a 2 GiB buffer (read + write bytes / time): the
    practical HBM ceiling on this machine, reported next to the datasheet peak."""
    a = torch.empty(mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * mib * 2 ** 20 / (ms * 1e-3) / 1e9


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--cpu-sample-n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and adjoint measurements")
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "TRACE_DIR"),
                    help="write profiles/ summaries from rocprofv3 runs of this script (no GPU needed)")
    args = ap.parse_args()
    if args.summarize_profiles:
        return summarize_profiles(*args.summarize_profiles, n=args.n)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} (WORLD_SIZE={world}) is not supported: "
              "the evaluation runs on a single MI355X and has no multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1501_04438_amd as gs
    import workloads

    dev = "cuda:0"
    torch.cuda.set_device(0)
    n = args.n
    prob = workloads.config2(n)
    # compiled launch variants (tuned for this size), so that the rocprofv3 runs of this
    # script profile exactly the kernels the timed loop runs
    plan = gs.Plan("coulomb3d", n=n, L=prob.L, eps=1e-14)
    rho = torch.from_numpy(prob.rho).to(dev)
    u = torch.empty_like(rho)
    print(f"# plan: n={n} Q={plan.info['Q']} spectrum assembly {plan.info['assembly_ms']:.3f} ms "
          f"({plan.info['assembly_gflop']:.2f} GFLOP)", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        plan.eval(rho, out=u)
    torch.cuda.synchronize()

    K = args.steps
    steps = plan.steps()                       # pass id of every launch of one evaluation
    S = len(steps)
    # HIP events without the system-scope fence (a timing-only event; with the fence every
    # record writes back and invalidates the caches), recorded by the library on the stream
    # the passes are launched on.  Each record still costs the stream a few microseconds, so
    # the per-pass breakdown comes from its own loop with an event after every pass, and the
    # timed loop records events only around the launches of the dominant kernel.
    hip = HipEvents()
    ev = [[hip.create() for _ in range(S + 1)] for _ in range(K)]

    def marked(p):
        """Events of each step's row only before and after the launches of pass p."""
        ds = [i for i, q in enumerate(steps) if q == p]
        return ds, [[row[j] if (j in ds or j - 1 in ds) else None for j in range(S + 1)] for row in ev]

    def pass_time(ds):
        return float(np.mean([sum(hip.elapsed(ev[s][i], ev[s][i + 1]) for i in ds) for s in range(K)]))

    # an event after every pass: the dominant pass, and the whole-evaluation GPU time with
    # those events in the chain
    for s in range(K):
        plan.eval_events(rho, u, ev[s])
    torch.cuda.synchronize()
    full_ms = {p: pass_time(marked(p)[0]) for p in sorted(set(steps))}
    per_step = [hip.elapsed(ev[s][0], ev[s][S]) for s in range(K)]
    gpu_ms = float(np.mean(per_step))
    dom = max(full_ms, key=full_ms.get)
    # every other pass with events around its own launches only
    pass_ms = {}
    for p in sorted(set(steps)):
        if p == dom:
            continue
        ds, marks = marked(p)
        for s in range(K):
            plan.eval_events(rho, u, marks[s])
        torch.cuda.synchronize()
        pass_ms[p] = pass_time(ds)
    # the timed region: K evaluations, events only around the launches of the dominant
    # kernel (its duration, measured live)
    dsteps, marks = marked(dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(K):
        plan.eval_events(rho, u, marks[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_step = wall / K * 1e3
    dom_ms = pass_time(dsteps)
    pass_ms[dom] = dom_ms
    hip.destroy([e for row in ev for e in row])
    value = n ** 3 / (wall / K) / 1e6
    # the same K evaluations, one library call each (no events)
    t0 = time.perf_counter()
    for _ in range(K):
        plan.eval(rho, out=u)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) / K * 1e3

    nb = pass_bytes(n)
    achieved = nb[dom] / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(PASS_NAMES[dom])
    passes = {PASS_NAMES[p]: {"ms": round(pass_ms[p], 5), "ms_all_pass_events": round(full_ms[p], 5),
                              "launches": steps.count(p), "alg_bytes": nb[p],
                              "GB_s": round(nb[p] / (pass_ms[p] * 1e-3) / 1e9, 1)} for p in sorted(pass_ms)}
    total_bytes = sum(nb.values())

    # accuracy of this very output against stored oracle samples
    acc = None
    gpath = os.path.join(ROOT, "tests", "golden", f"oracle_c2_coulomb3d_{n}.npz")
    if os.path.exists(gpath):
        g = np.load(gpath)
        plan.eval(rho, out=u)
        uh = u.cpu().numpy()
        acc = float(np.max(np.abs(uh[tuple(g["idx"].T)] - g["u"])) / float(g["umax"]))

    out = {
        "metric": "Mpts/s per potential eval, 3D Coulomb 256^3 FP64 @<=1e-12",
        "value": round(value, 1), "unit": "Mpts/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"coulomb3d_{n}_triaxial_plus_8_gaussian_mixture_L10", "n": n, "L": prob.L,
                   "kernel": "coulomb3d", "eps": 1e-14, "delta_rel": 1e-4, "Q": plan.info["Q"],
                   "slab_planes": plan.info["slab_planes"], "launches": S,
                   "launch_variants": {"hint_bits": plan.info["hint_bits"],
                                       "fused_grid_mult": plan.info["fused_grid_mult"],
                                       "autotuned": plan.info["tuned"]}},
        "roofline": {"bound": "hbm", "kernel": PASS_NAMES[dom], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "ms": round(dom_ms, 5)},
        "ms_per_eval_without_events": round(plain_ms, 5),
        "gpu_ms_per_eval_all_pass_events": round(gpu_ms, 5),
        "gpu_ms_per_eval_all_pass_events_median": round(float(np.median(per_step)), 5),
        "eval_alg_bytes": total_bytes,
        "eval_GB_s": round(total_bytes / (ms_step * 1e-3) / 1e9, 1),
        "eval_frac_hbm": round(total_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "passes": passes,
        "max_rel_err_vs_oracle_samples": acc,
        "assembly": {"ms": round(plan.info["assembly_ms"], 4), "gflop": round(plan.info["assembly_gflop"], 3),
                     "tflops": round(plan.info["assembly_gflop"] / max(plan.info["assembly_ms"], 1e-9), 2),
                     "frac_fp64_mfma": round(plan.info["assembly_gflop"] / max(plan.info["assembly_ms"], 1e-9)
                                             / FP64_MFMA_PEAK_TFLOPS, 4)},
        "paper_context": {"value": 0.850, "unit": "Mpts/s", "hardware": "Xeon E5540 2.53 GHz, Fortran, ifort -O3",
                          "workload": "3D Coulomb 256^3, isotropic Gaussian sigma=1.2 on [-8,8]^3 (Table 1)"},
    }

    out["copy_GB_s"] = round(copy_bandwidth(torch), 1)
    if not args.no_extras:
        dg = dgemm_tflops(torch)
        out["dgemm_TFLOPs"] = round(dg, 2)
        out["assembly"]["frac_measured_dgemm"] = round(out["assembly"]["tflops"] / dg, 4)
    if not args.no_extras:
        out["autotuned_plan"] = autotuned_figures(gs, torch, plan, rho, K)
        out["adjoint"] = adjoint_figures(gs, torch, workloads, plan, rho, K, ms_step)
        out["batched"] = batched_figures(gs, torch, workloads)
        out["other_workloads"] = other_figures(gs, torch, workloads)
        out["graph_replay"] = graph_figures(gs, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_n)
    print(json.dumps(out), flush=True)
    return 0


def autotuned_figures(gs, torch, plan, rho, K):
    """The plan autotuner on the headline grid (cache hints, fused-pass grid rounds, the
    tile shapes of the passes and the fused pass's radix plan): its choice, and its
    evaluation time next to the compiled defaults' (both timed here with events on the
    current stream; the same bits unless it chose a radix-plan variant, tile bits 8-12,
    which agrees to rounding: its largest difference is reported)."""
    tuned = gs.Plan("coulomb3d", n=plan.n, L=plan.L, eps=1e-14, autotune=True)
    info = tuned.query()
    u = torch.empty_like(rho)

    def timed(p):
        for _ in range(3):
            p.eval(rho, out=u)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(K):
            p.eval(rho, out=u)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K

    ms_default, ms_tuned = timed(plan), timed(tuned)
    res = {"hint_bits": info["hint_bits"], "fused_grid_mult": info["fused_grid_mult"],
           "tile_variants": info["tile_variants"], "candidates_timed": info["tune_candidates"],
           "ms_tuned": round(ms_tuned, 5), "ms_default": round(ms_default, 5),
           "radix_variant": bool(info["tile_variants"] & (31 << 8))}
    ut, ud = tuned.eval(rho), plan.eval(rho)
    res["bitwise_equal"] = bool(torch.equal(ut, ud))
    res["max_rel_diff_vs_default"] = float((ut - ud).abs().max() / ud.abs().max())
    tuned.close()
    return res


def graph_figures(gs, torch, reps: int = 200):
    """An evaluation captured in a HIP graph (torch.cuda.CUDAGraph around plan.eval) and
    replayed, against the same evaluation launched eagerly: the launch cost that small grids
    pay (the same bits either way)."""
    res = {}
    for kernel, n, L in (("coulomb3d", 32, 8.0), ("coulomb2d", 192, 12.0), ("coulomb3d", 64, 8.0),
                         ("coulomb3d", 128, 10.0)):
        d = 2 if kernel.endswith("2d") else 3
        plan = gs.Plan(kernel, n=n, L=L, eps=1e-14)
        x = torch.randn((n,) * d, dtype=torch.float64, device="cuda:0")
        u = torch.empty_like(x)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                plan.eval(x, out=u)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.eval(x, out=u)

        def timed(fn):
            for _ in range(5):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        ms_eager = timed(lambda: plan.eval(x, out=u))
        ue = u.clone()
        ms_graph = timed(g.replay)
        res[f"{kernel}_{n}"] = {"ms_eager": round(ms_eager, 5), "ms_graph": round(ms_graph, 5),
                                "launches": len(plan.steps()), "same_bits": bool(torch.equal(u, ue))}
        del g
        plan.close()
    return res


def other_workloads_bytes(d: int, n: int) -> int:
    """Algorithmic bytes of one evaluation (2D: P1, fused P3 along y, P5)."""
    if d == 3:
        return sum(pass_bytes(n).values())
    return 16 * n * n + 64 * (n + 1) * n + 8 * (n + 1) ** 2


def grid_chain_bytes(nx: int, ny: int, nz: int) -> int:
    """Algorithmic bytes of the five 3D passes on a grid of nx x ny x nz points (each axis its
    own n): X1 [z][kx][y] and X2 [kx][ky][z] complex, the spectrum octant once."""
    real = 8 * nx * ny * nz
    x1 = 16 * (nx + 1) * ny * nz
    x2 = 32 * (nx + 1) * ny * nz
    spec = 8 * (nx + 1) * (ny + 1) * (nz + 1)
    return (real + x1) + (x1 + x2) + (2 * x2 + spec) + (x2 + x1) + (x1 + real)


def padding3_bytes(n: int) -> int:
    """Padding to B_3 of an n^3 grid: the chain on the m = 3n/2 transform grid, whose x-forward
    pass reads the n^3 density itself, whose y-inverse pass runs for the planes z < n only and
    whose x-inverse pass reads the rows y < n of those planes and writes the n^3 potential (no
    copies of the transform grid's size)."""
    m = 3 * n // 2
    x1 = 16 * (m + 1) * m * m       # [z][kx][y] complex
    x2 = 32 * (m + 1) * m * m       # [kx][ky][z] complex
    spec = 8 * (m + 1) ** 3
    f = n / m
    return round(8 * n ** 3 + x1 + (x1 + x2) + (2 * x2 + spec) + (x2 + x1) * f + x1 * f * f + 8 * n ** 3)


def other_figures(gs, torch, workloads, reps: int = 20):
    """Evaluation throughput of the other workloads: 2D Poisson, Coulomb and Davey-Stewartson at 2048^2,
    2D Poisson and Coulomb at 1024^2, 3D dipolar at 128^3, 3D Coulomb at 128^3, and the rectangular boxes of the
    anisotropic tables (3D 96^3 with gamma = 8, 2D 192^2 with gamma = 16); working
    sets partly resident in the Infinity Cache, so their bandwidth fraction can
    exceed what HBM alone allows.  Then the widened rows at the headline size: the
    inverse power r^-1.5, the unpadded-grid Laplacian, padding to B_3, a 128 x 256 x 512
    grid with one step and a 320^3 grid (radix-5 stages)."""
    res = {}
    cases = [("poisson2d_2048", workloads.config3_2d("poisson2d", 2048), {"eps": 1e-13}),
             ("coulomb2d_2048", workloads.config3_2d("coulomb2d", 2048), {}),
             ("davey_stewartson2d_2048", workloads.config3_2d("davey_stewartson2d", 2048), {"eps": 1e-13}),
             ("poisson2d_1024", workloads.config3_2d("poisson2d", 1024), {"eps": 1e-13}),
             ("coulomb2d_1024", workloads.config3_2d("coulomb2d", 1024), {}),
             ("dipolar3d_128", workloads.config3_dipolar(128), None),
             ("coulomb3d_128", workloads.config2(128), {}),
             ("rect_coulomb3d_96_gamma8", workloads.rect_box(3, 8.0), {}),
             ("rect_coulomb2d_192_gamma16", workloads.rect_box(2, 16.0), {})]
    # the widened rows at the headline size: inverse power, the two fidelity variants, a grid
    # with its own n per axis (one step h = 1/25.6) and a length with a factor 5
    c2 = workloads.config2(256)
    ext = [("inverse_power3d_256_beta1.5", workloads.Problem("inverse_power", 3, 256, c2.L, c2.rho),
            {"beta": 1.5, "d": 3}, sum(pass_bytes(256).values())),
           ("unpadded_laplacian_coulomb3d_256", c2, {"laplacian": "unpadded"}, sum(pass_bytes(256).values())),
           ("padding3_coulomb3d_256", c2, {"padding": 3}, padding3_bytes(256)),
           ("per_axis_coulomb3d_128x256x512",
            workloads.Problem("coulomb3d", 3, (128, 256, 512), (5.0, 10.0, 20.0),
                              workloads.gaussian((128, 256, 512), (5.0, 10.0, 20.0), 3, sigma=2.0)),
            {}, grid_chain_bytes(512, 256, 128)),
           ("radix5_coulomb3d_320", workloads.config2(320), {}, sum(pass_bytes(320).values()))]
    cases = [(a, b, c, None) for a, b, c in cases] + ext
    for name, p, kw, nbytes in cases:
        if kw is None:
            kw = {"dipole": (p.extra["n"], p.extra["m"])}
        plan = gs.Plan(p.kernel, n=p.n, L=p.L, autotune=True, **kw)
        rho = torch.from_numpy(p.rho).to("cuda:0")
        u = torch.empty_like(rho)
        for _ in range(3):
            plan.eval(rho, out=u)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            plan.eval(rho, out=u)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        pts = 1
        for v in plan.shape:
            pts *= int(v)
        b = nbytes if nbytes is not None else other_workloads_bytes(p.d, p.n)
        res[name] = {"ms": round(ms, 4), "Mpts_s": round(pts / ms / 1e3, 1), "alg_GB_s": round(b / ms / 1e6, 1),
                     "frac_hbm": round(b / ms / 1e6 / HBM_PEAK_GBS, 4),
                     "hint_bits": plan.info["hint_bits"], "fused_grid_mult": plan.info["fused_grid_mult"],
                     "tile_variants": plan.info["tile_variants"]}
        plan.close()
    return res


def adjoint_figures(gs, torch, workloads, plan, rho, K, eval_ms):
    """The adjoint chain alone; energy + rho-gradient through autograd (gs.energy: the energy
    summed inside the evaluation's last pass, the gradient cell * u, which autograd forms with
    one more pass over the grid) and directly (plan.energy_and_gradient: the last pass writes
    cell * u and sums the energy); and the differentiation
    workload: the energy of the 8-component mixture on the same grid with its gradient with
    respect to all 40 mixture parameters (gs.mixture_energy: density, evaluation with energy
    and gradient reduction in library kernels), each against the plain evaluation."""
    g = torch.empty_like(rho)
    for _ in range(2):
        plan.eval_backward(rho, out=g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        plan.eval_backward(rho, out=g)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / K
    r = rho.clone().requires_grad_(True)
    E = gs.energy(r, plan)
    E.backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(3, K // 5)
    for _ in range(reps):
        r.grad = None
        E = gs.energy(r, plan)
        E.backward()
    torch.cuda.synchronize()
    dte = (time.perf_counter() - t0) / reps
    gbuf = torch.empty_like(rho)
    for _ in range(2):
        plan.energy_and_gradient(rho, out=gbuf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        plan.energy_and_gradient(rho, out=gbuf)
    torch.cuda.synchronize()
    dtd = (time.perf_counter() - t0) / K
    m = workloads.config5_mixture()
    t = lambda x: torch.tensor(x, dtype=torch.float64, device="cuda:0", requires_grad=True)
    a, mu, s = t(m.a), t(m.mu), t(m.sigma)

    def mixture_step():
        E = gs.mixture_energy(a, mu, s, plan)
        return torch.autograd.grad(E, (a, mu, s))

    for _ in range(2):
        mixture_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mixture_step()
    torch.cuda.synchronize()
    dtm = (time.perf_counter() - t0) / reps
    n3 = rho.numel()
    return {"backward_Mpts_s": round(n3 / dt / 1e6, 1), "backward_ms": round(dt * 1e3, 4),
            "energy_and_grad_Mpts_s": round(n3 / dte / 1e6, 1), "energy_and_grad_ms": round(dte * 1e3, 4),
            "energy_and_grad_over_eval": round(dte * 1e3 / eval_ms, 3),
            "energy_and_grad_direct_ms": round(dtd * 1e3, 4),
            "energy_and_grad_direct_over_eval": round(dtd * 1e3 / eval_ms, 3),
            "mixture_energy_and_40_param_grads_ms": round(dtm * 1e3, 4),
            "mixture_energy_and_40_param_grads_Mpts_s": round(n3 / dtm / 1e6, 1),
            "mixture_over_eval": round(dtm * 1e3 / eval_ms, 3)}


def batched_figures(gs, torch, workloads, reps: int = 10):
    """64 seeded mixtures on uneven grids (32..128 points per axis): the batch
    schedules against 64 plain solves (plan.eval one after the other)."""
    probs = [workloads.materialise(p) for p in workloads.config4(64)]
    plans = [gs.Plan("coulomb3d", n=p.n, L=p.L, eps=1e-14) for p in probs]
    rhos = [torch.from_numpy(p.rho).to("cuda:0") for p in probs]
    pts = sum(p.n ** 3 for p in probs)
    ref = [pl.eval(r) for pl, r in zip(plans, rhos)]
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    outs = [torch.empty_like(r) for r in rhos]
    alg = sum(sum(pass_bytes(p.n).values()) for p in probs)
    res = {"problems": len(probs), "points": pts, "sizes": sorted({p.n for p in probs}), "reps": reps,
           "alg_bytes": alg}
    ms = timed(lambda: [pl.eval(r, out=o) for pl, r, o in zip(plans, rhos, outs)])
    res["single_solves"] = {"ms": round(ms, 4), "Mpts_s": round(pts / ms / 1e3, 1),
                            "alg_GB_s": round(alg / ms / 1e6, 1), "frac_hbm": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}
    equal = all(torch.equal(o, r) for o, r in zip(outs, ref))
    for name, kw in [("sequential", dict(schedule="sequential")),
                     ("sequential_graph", dict(schedule="sequential", graph=True)),
                     ("phased", dict(schedule="phased")),
                     ("sized", dict(schedule="sized")),
                     ("sized_graph", dict(schedule="sized", graph=True)),
                     ("concurrent", dict(schedule="concurrent")),
                     ("concurrent_graph", dict(schedule="concurrent", graph=True)),
                     ("streams", dict(schedule="streams")),
                     ("streams_graph", dict(schedule="streams", graph=True)),
                     ("queue", dict(schedule="queue")),
                     ("queue_graph", dict(schedule="queue", graph=True)),
                     ("auto_graph", dict(schedule="auto", graph=True))]:
        b = gs.Batch(plans, **kw)
        outs = [torch.empty_like(r) for r in rhos]
        ms = timed(lambda: b.eval(rhos, outs))
        equal = equal and all(torch.equal(o, r) for o, r in zip(outs, ref))
        info = b.info
        res[name] = {"ms": round(ms, 4), "Mpts_s": round(pts / ms / 1e3, 1), "schedule": info["schedule"],
                     "tiles_per_task": info["tiles_per_task"], "tasks": info["num_tasks"],
                     "alg_GB_s": round(alg / ms / 1e6, 1), "frac_hbm": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}
        if name.startswith("auto"):
            res[name]["candidates_timed"] = info["candidates"]
        b.close()
    best = min((v["ms"], k) for k, v in res.items() if isinstance(v, dict) and k != "single_solves")
    res["best"] = best[1]
    res["speedup_vs_single_solves"] = round(res["single_solves"]["ms"] / best[0], 2)
    res["bitwise_equal_to_single"] = bool(equal)
    return res


if __name__ == "__main__":
    sys.exit(main())
