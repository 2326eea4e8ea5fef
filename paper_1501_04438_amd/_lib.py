"""ctypes declarations of the C ABI in include/gs.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs.so")

KERNELS = {"coulomb3d": 0, "coulomb2d": 1, "poisson2d": 2, "dipolar3d": 3, "gaussian_sum": 4,
           "davey_stewartson2d": 5, "inverse_power": 6}
KERNEL_DIM = {"coulomb3d": 3, "coulomb2d": 2, "poisson2d": 2, "dipolar3d": 3, "davey_stewartson2d": 2}

GS_OK = 0
STATUS = {0: "GS_OK", 1: "GS_ERR_INVALID_ARG", 2: "GS_ERR_UNSUPPORTED_SIZE", 3: "GS_ERR_ACCURACY",
          4: "GS_ERR_OUT_OF_MEMORY", 5: "GS_ERR_NO_DEVICE", 6: "GS_ERR_HIP"}
PLAN_HOST_ONLY = 1
PLAN_HOST_ASSEMBLY = 2
PLAN_AUTOTUNE = 4
PLAN_NO_WORKSPACE = 8
PLAN_UNPADDED_LAPLACIAN = 16
PLAN_PAD3 = 32


class GSOptions(C.Structure):
    _fields_ = [("delta_rel", C.c_double), ("dipole_n", C.c_double * 3), ("dipole_m", C.c_double * 3),
                ("gs_w", C.POINTER(C.c_double)), ("gs_tau", C.POINTER(C.c_double)), ("gs_q", C.c_int),
                ("stream", C.c_void_p), ("device", C.c_int), ("flags", C.c_int), ("slab_planes", C.c_int),
                ("slab_streams", C.c_int), ("beta", C.c_double), ("tile_variants", C.c_int),
                ("launch_hints", C.c_int)]


class GSPlanInfo(C.Structure):
    _fields_ = [("kernel", C.c_int), ("d", C.c_int), ("n", C.c_int64), ("L", C.c_double), ("eps", C.c_double),
                ("delta", C.c_double), ("S", C.c_int), ("Q", C.c_int), ("A0", C.c_double), ("c2", C.c_double),
                ("spectrum_bytes", C.c_size_t), ("workspace_bytes", C.c_size_t), ("assembly_ms", C.c_double),
                ("assembly_gflop", C.c_double), ("host_only", C.c_int), ("slab_planes", C.c_int),
                ("num_steps", C.c_int), ("slab_streams", C.c_int), ("x2_planes", C.c_int), ("tuned", C.c_int), ("hint_bits", C.c_int), ("fused_grid_mult", C.c_int),
                ("tune_candidates", C.c_int), ("tuned_ms", C.c_double), ("L_axes", C.c_double * 3),
                ("beta", C.c_double), ("n_axes", C.c_int64 * 3), ("tile_variants", C.c_int),
                ("padding", C.c_int)]


SCHEDULES = {"auto": 0, "queue": 1, "phased": 2, "sequential": 3, "sized": 4, "concurrent": 5, "streams": 6}


class GSBatchOptions(C.Structure):
    _fields_ = [("schedule", C.c_int), ("tiles_per_task", C.c_int), ("grid", C.c_int), ("use_graph", C.c_int),
                ("stream", C.c_void_p)]


class GSBatchInfo(C.Structure):
    _fields_ = [("count", C.c_int), ("points", C.c_double), ("schedule", C.c_int), ("tiles_per_task", C.c_int),
                ("grid", C.c_int), ("use_graph", C.c_int), ("num_tasks", C.c_int), ("tasks_per_pass", C.c_int * 6),
                ("autotuned", C.c_int), ("candidates", C.c_int), ("tuned_ms", C.c_double),
                ("wait_timeouts", C.c_int), ("num_queues", C.c_int), ("local_queues", C.c_int)]


# name -> (restype, argtypes); every symbol declared in include/gs.h
SIGNATURES = {
    "gs_options_default": (None, [C.POINTER(GSOptions)]),
    "gs_plan_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.POINTER(C.c_int64),
                                 C.POINTER(C.c_double), C.c_double, C.POINTER(GSOptions)]),
    "gs_plan_destroy": (C.c_int, [C.c_void_p]),
    "gs_plan_query": (C.c_int, [C.c_void_p, C.POINTER(GSPlanInfo)]),
    "gs_plan_table": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int]),
    "gs_plan_factors": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_size_t]),
    "gs_plan_factors_axis": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_size_t]),
    "gs_plan_spectrum": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_size_t]),
    "gs_plan_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gs_eval": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gs_eval_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gs_eval_batch": (C.c_int, [C.c_int, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    "gs_batch_options_default": (None, [C.POINTER(GSBatchOptions)]),
    "gs_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_void_p),
                                  C.POINTER(GSBatchOptions)]),
    "gs_batch_eval": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    "gs_batch_query": (C.c_int, [C.c_void_p, C.POINTER(GSBatchInfo)]),
    "gs_eval_energy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gs_eval_energy_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gs_mixture_density": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "gs_mixture_gradient": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_double, C.c_void_p]),
    "gs_eval_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "gs_batch_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "gs_batch_destroy": (C.c_int, [C.c_void_p]),
    "gs_eval_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "gs_eval_events": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p), C.c_int]),
    "gs_plan_steps": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.c_int]),
    "gs_plan_buffer": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_size_t]),
    "gs_status_string": (C.c_char_p, [C.c_int]),
    "gs_last_error": (C.c_char_p, []),
    "gs_device_count": (C.c_int, []),
    "gs_supported_sizes": (C.c_int, [C.c_int, C.POINTER(C.c_int64), C.c_int]),
}

_lib = None


class GSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded library; raises if libgs.so was not built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1501_04438_amd.build` "
                              "(or __graft_entry__.build()); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != GS_OK:
        raise GSError(status, lib().gs_last_error().decode())
