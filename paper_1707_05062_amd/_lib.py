"""ctypes declarations for libkohler.so (the C ABI of include/kohler.h). Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkohler.so")

OK, E_ARG, E_RANGE, E_CAPACITY, E_NOMEM, E_DEVICE, E_BUSY, E_CANCELED = 0, -1, -2, -3, -4, -5, -6, -7
U8, U16 = 1, 2
MAX_M_U16 = 10200

# every symbol include/kohler.h declares
EXPORTS = (
    "kohler_create", "kohler_destroy", "kohler_strerror", "kohler_curve", "kohler_curve_async",
    "kohler_curve_batch", "kohler_curve_noalloc", "kohler_curve_nbhd_async", "kohler_set_plan", "kohler_get_plan", "kohler_autotune", "kohler_segment",
    "kohler_class_stats", "kohler_mean_image", "kohler_top_thresholds",
    "kohler_server_create", "kohler_server_destroy", "kohler_server_submit", "kohler_server_submit_labels",
    "kohler_server_poll",
    "kohler_server_wait", "kohler_server_cancel", "kohler_server_pause", "kohler_server_stats",
)


class _Struct(ctypes.Structure):
    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "pad"}


NBHD_OFFSETS, NBHD_HEX6 = 1, 2
NBHD_MAX_HALF = 16


class Nbhd(_Struct):
    _fields_ = [("kind", ctypes.c_int32), ("n_half", ctypes.c_int32),
                ("half_dy", ctypes.c_int32 * NBHD_MAX_HALF), ("half_dx", ctypes.c_int32 * NBHD_MAX_HALF)]


class Plan(_Struct):
    _fields_ = [("form", ctypes.c_int32), ("band", ctypes.c_int32), ("block", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("px_per_lane", ctypes.c_int32),
                ("replicas", ctypes.c_int32), ("copies", ctypes.c_int32), ("acc_split", ctypes.c_int32)]


class ServerConfig(_Struct):
    _fields_ = [("dtype", ctypes.c_int32), ("M", ctypes.c_int32), ("nbhd", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("lanes", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("thr_capacity", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32), ("label_t0", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64)]


class RequestInfo(_Struct):
    _fields_ = [("status", ctypes.c_int32), ("n_thresholds", ctypes.c_int32), ("t0", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("graph", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("t_submit_ns", ctypes.c_int64), ("t_launch_ns", ctypes.c_int64),
                ("t_issued_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


class ServerCounters(_Struct):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "submitted", "completed", "refused", "cancelled", "launches", "graph_launches",
        "batched_launches", "graphs_built", "max_batch_seen", "peak_inflight", "arena_bytes",
        "arena_peak_bytes", "slot_state_bytes")]


_lib = None


def load(path: str = LIB_PATH):
    """Load and declare the library. Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_1707_05062_amd.build` "
            "(the contrast curve runs only through the HIP library)")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    i64p, i32p, f64p = ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)

    lib.kohler_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.kohler_create.restype = ctypes.c_int
    lib.kohler_destroy.argtypes = [vp]
    lib.kohler_destroy.restype = None
    lib.kohler_strerror.argtypes = [ctypes.c_int]
    lib.kohler_strerror.restype = ctypes.c_char_p
    lib.kohler_curve.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, i32, i32, i64p, i64p, f64p,
                                 i32p, i32, i32p, i32p]
    lib.kohler_curve.restype = ctypes.c_int
    lib.kohler_curve_async.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, i32, i32, vp, vp, vp,
                                       vp, i32, vp, vp, vp, vp]
    lib.kohler_curve_async.restype = ctypes.c_int
    lib.kohler_curve_batch.argtypes = [vp, i32, ctypes.POINTER(vp), i64p, i64p, i64p, ctypes.c_int,
                                       i32, i32, vp, vp, vp, vp, i32, vp, vp, vp, vp]
    lib.kohler_curve_batch.restype = ctypes.c_int
    lib.kohler_curve_noalloc.argtypes = [vp, ctypes.c_int, i64, i64, i64, i32, i32, vp, vp, vp, vp, i32, vp, vp,
                                         vp, ctypes.POINTER(Plan), vp]
    lib.kohler_curve_noalloc.restype = ctypes.c_int
    lib.kohler_curve_nbhd_async.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, i32, ctypes.POINTER(Nbhd), i32,
                                            vp, vp, vp, vp, i32, vp, vp, vp, vp]
    lib.kohler_curve_nbhd_async.restype = ctypes.c_int
    lib.kohler_set_plan.argtypes = [vp, ctypes.c_int, i32, i32, ctypes.POINTER(Plan)]
    lib.kohler_set_plan.restype = ctypes.c_int
    lib.kohler_get_plan.argtypes = [vp, ctypes.c_int, i64, i64, i32, i32, ctypes.POINTER(Plan)]
    lib.kohler_get_plan.restype = ctypes.c_int
    lib.kohler_autotune.argtypes = [vp, i32, ctypes.POINTER(vp), i64p, i64p, i64p, ctypes.c_int, i32,
                                    i32, i32, ctypes.POINTER(Plan), f64p]
    lib.kohler_autotune.restype = ctypes.c_int
    lib.kohler_segment.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, i32, vp, vp, i32, vp, ctypes.c_int,
                                   i64, vp]
    lib.kohler_segment.restype = ctypes.c_int
    lib.kohler_class_stats.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, i32, vp, vp, i32, vp, vp, vp, vp]
    lib.kohler_class_stats.restype = ctypes.c_int
    lib.kohler_mean_image.argtypes = [vp, vp, ctypes.c_int, i64, i64, i64, i32, vp, vp, i32, vp, vp, i64, vp]
    lib.kohler_mean_image.restype = ctypes.c_int
    lib.kohler_top_thresholds.argtypes = [vp, vp, vp, i32, vp, vp, i32, i32, vp, vp, vp]
    lib.kohler_top_thresholds.restype = ctypes.c_int
    u64 = ctypes.c_uint64
    lib.kohler_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.kohler_server_create.restype = ctypes.c_int
    lib.kohler_server_destroy.argtypes = [vp]
    lib.kohler_server_destroy.restype = None
    lib.kohler_server_submit.argtypes = [vp, vp, i64, i64, i64, ctypes.POINTER(u64)]
    lib.kohler_server_submit.restype = ctypes.c_int
    lib.kohler_server_submit_labels.argtypes = [vp, vp, i64, i64, i64, vp, i64, ctypes.POINTER(u64)]
    lib.kohler_server_submit_labels.restype = ctypes.c_int
    lib.kohler_server_poll.argtypes = [vp, u64]
    lib.kohler_server_poll.restype = ctypes.c_int
    lib.kohler_server_wait.argtypes = [vp, u64, vp, vp, vp, vp, i32, ctypes.POINTER(RequestInfo)]
    lib.kohler_server_wait.restype = ctypes.c_int
    lib.kohler_server_cancel.argtypes = [vp, u64]
    lib.kohler_server_cancel.restype = ctypes.c_int
    lib.kohler_server_pause.argtypes = [vp, i32]
    lib.kohler_server_pause.restype = ctypes.c_int
    lib.kohler_server_stats.argtypes = [vp, ctypes.POINTER(ServerCounters)]
    lib.kohler_server_stats.restype = ctypes.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().kohler_strerror(status).decode()
