"""ctypes declarations of the C ABI in include/mpk.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmpk.so")

MPK_OK, MPK_EINVAL, MPK_EBADCSR, MPK_ENOMEM, MPK_EHIP, MPK_EUNSUPPORTED, MPK_ETIMEOUT, \
    MPK_ENODEVICE = range(8)
STATUS_NAMES = {0: "MPK_OK", 1: "MPK_EINVAL", 2: "MPK_EBADCSR", 3: "MPK_ENOMEM", 4: "MPK_EHIP",
                5: "MPK_EUNSUPPORTED", 6: "MPK_ETIMEOUT", 7: "MPK_ENODEVICE"}
MPK_ORDER_ORIGINAL, MPK_ORDER_PLAN = 0, 1
MPK_REORDER_BFS, MPK_REORDER_NONE, MPK_REORDER_SUBLEVELS = 0, 1, 2
MPK_ROOT_AUTO = -1
MPK_SCHED_STEPS, MPK_SCHED_WAVE, MPK_SCHED_DIAG, MPK_SCHED_POWERS, MPK_SCHED_XCD = 0, 1, 2, 3, 4
MPK_DEVICE_CURRENT, MPK_DEVICE_NONE = -1, -2
MPK_MAX_RHS = 16

# every symbol the header declares
EXPORTS = [
    "mpk_plan_opts_default", "mpk_tune_default", "mpk_plan", "mpk_plan_destroy", "mpk_plan_tune",
    "mpk_plan_info", "mpk_plan_levels", "mpk_plan_schedule", "mpk_plan_schedule_xcd", "mpk_run", "mpk_run_recur",
    "mpk_run_baseline", "mpk_run_baseline_recur", "mpk_permute", "mpk_plan_sync",
    "mpk_set_allocator", "mpk_last_error", "mpk_version", "mpk_probe_load", "mpk_probe_load_xcd", "mpk_run_status", "mpk_run_noalloc",
    "mpk_plan_autotune", "mpk_graph_capture", "mpk_graph_launch", "mpk_graph_destroy",
    "mpk_run_poly", "mpk_run_baseline_poly", "mpk_cheb_time_coefficients", "mpk_combine_complex",
    "mpk_graph_capture_time_step", "mpk_plan_device", "mpk_plan_prepare",
]

c_i32p = ctypes.POINTER(ctypes.c_int32)
c_f64p = ctypes.POINTER(ctypes.c_double)


class CSRStruct(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("value_bits", ctypes.c_int), ("reorder", ctypes.c_int), ("order", ctypes.c_int),
                ("root", ctypes.c_int), ("device", ctypes.c_int), ("l2_bytes", ctypes.c_int64),
                ("mall_bytes", ctypes.c_int64), ("min_group_rows", ctypes.c_int),
                ("sublevel_root", ctypes.c_int)]


class Tune(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int), ("cache_bytes", ctypes.c_int64),
                ("cache_safety", ctypes.c_double), ("chunk_nnz", ctypes.c_int),
                ("lag", ctypes.c_int), ("workgroups", ctypes.c_int),
                ("spin_limit_us", ctypes.c_int64), ("seg_powers", ctypes.c_int),
                ("skip_ahead", ctypes.c_int), ("acquire_always", ctypes.c_int),
                ("dynamic_tickets", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_levels", ctypes.c_int32),
                ("max_level_rows", ctypes.c_int32), ("value_bits", ctypes.c_int32),
                ("reorder", ctypes.c_int32), ("order", ctypes.c_int32),
                ("matrix_bytes", ctypes.c_int64),
                ("plan_ms", ctypes.c_double), ("device", ctypes.c_int32),
                ("sliced_layout", ctypes.c_int32), ("sliced_entries", ctypes.c_int64),
                ("sublevel_root", ctypes.c_int32), ("max_sublevels", ctypes.c_int32),
                ("l2_bytes", ctypes.c_int64), ("mall_bytes", ctypes.c_int64),
                ("min_group_rows", ctypes.c_int32), ("sliced_col_bits", ctypes.c_int32),
                ("fingerprint", ctypes.c_uint64)]


class SchedInfo(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("n_chunks", ctypes.c_int32), ("n_groups", ctypes.c_int32),
                ("n_tasks", ctypes.c_int32), ("n_steps", ctypes.c_int32), ("lag", ctypes.c_int32),
                ("max_reach", ctypes.c_int32),
                ("window_bytes", ctypes.c_double), ("build_ms", ctypes.c_double),
                ("n_queues", ctypes.c_int32), ("n_deps", ctypes.c_int32)]


_lib = None


def load():
    """Load libmpk.so; raise (never fall back) when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2405_12525_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    st = ctypes.c_int
    lib.mpk_plan_opts_default.argtypes = [ctypes.POINTER(PlanOpts)]
    lib.mpk_plan_opts_default.restype = None
    lib.mpk_tune_default.argtypes = [ctypes.POINTER(Tune)]
    lib.mpk_tune_default.restype = None
    lib.mpk_plan.argtypes = [ctypes.POINTER(CSRStruct), ctypes.POINTER(PlanOpts),
                             ctypes.POINTER(ctypes.c_void_p)]
    lib.mpk_plan.restype = st
    lib.mpk_plan_device.argtypes = [ctypes.POINTER(CSRStruct), ctypes.POINTER(PlanOpts),
                                    ctypes.POINTER(ctypes.c_void_p)]
    lib.mpk_plan_device.restype = st
    lib.mpk_plan_destroy.argtypes = [P]
    lib.mpk_plan_destroy.restype = None
    lib.mpk_plan_tune.argtypes = [P, ctypes.POINTER(Tune)]
    lib.mpk_plan_tune.restype = st
    lib.mpk_plan_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
    lib.mpk_plan_info.restype = st
    lib.mpk_plan_levels.argtypes = [P, P, P]
    lib.mpk_plan_levels.restype = st
    lib.mpk_plan_schedule.argtypes = [P, ctypes.c_int, ctypes.POINTER(SchedInfo), P, P, P, P, P, P]
    lib.mpk_plan_schedule.restype = st
    lib.mpk_plan_schedule_xcd.argtypes = [P, ctypes.c_int, P, P, P, P, P]
    lib.mpk_plan_schedule_xcd.restype = st
    lib.mpk_plan_prepare.argtypes = [P, ctypes.c_int, ctypes.c_int]
    lib.mpk_plan_prepare.restype = st
    lib.mpk_run.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, P]
    lib.mpk_run.restype = st
    lib.mpk_run_recur.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, P, P, P, P]
    lib.mpk_run_recur.restype = st
    lib.mpk_run_baseline.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, P]
    lib.mpk_run_baseline.restype = st
    lib.mpk_run_baseline_recur.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, P, P, P, P]
    lib.mpk_run_baseline_recur.restype = st
    for f in (lib.mpk_run_poly, lib.mpk_run_baseline_poly):
        f.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, P]
        f.restype = st
    lib.mpk_cheb_time_coefficients.argtypes = [ctypes.c_int, ctypes.c_double, P, P, P, P, P]
    lib.mpk_cheb_time_coefficients.restype = st
    lib.mpk_graph_capture_time_step.argtypes = [P, P, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                                ctypes.c_int, P, P, P, ctypes.POINTER(P)]
    lib.mpk_graph_capture_time_step.restype = st
    lib.mpk_combine_complex.argtypes = [P, P, ctypes.c_int, P, P]
    lib.mpk_combine_complex.restype = st
    lib.mpk_permute.argtypes = [P, ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int, P]
    lib.mpk_permute.restype = st
    lib.mpk_plan_sync.argtypes = [P]
    lib.mpk_plan_sync.restype = st
    lib.mpk_probe_load.argtypes = [P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, P]
    lib.mpk_probe_load.restype = st
    lib.mpk_probe_load_xcd.argtypes = [P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       P, P, P]
    lib.mpk_probe_load_xcd.restype = st
    lib.mpk_run_status.argtypes = [P, P, P]
    lib.mpk_run_status.restype = st
    lib.mpk_run_noalloc.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, P, P]
    lib.mpk_run_noalloc.restype = st
    lib.mpk_plan_autotune.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, P, ctypes.POINTER(Tune),
                                      ctypes.POINTER(ctypes.c_double)]
    lib.mpk_plan_autotune.restype = st
    lib.mpk_graph_capture.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, P, P, P,
                                      ctypes.POINTER(ctypes.c_void_p)]
    lib.mpk_graph_capture.restype = st
    lib.mpk_graph_launch.argtypes = [P, P]
    lib.mpk_graph_launch.restype = st
    lib.mpk_graph_destroy.argtypes = [P]
    lib.mpk_graph_destroy.restype = None
    lib.mpk_set_allocator.argtypes = [P, P, P]
    lib.mpk_set_allocator.restype = st
    lib.mpk_last_error.argtypes = []
    lib.mpk_last_error.restype = ctypes.c_char_p
    lib.mpk_version.argtypes = []
    lib.mpk_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


class MPKError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


def check(status: int):
    if status != MPK_OK:
        msg = load().mpk_last_error().decode(errors="replace")
        raise MPKError(status, msg)
