"""ctypes declarations for libkohler.so (the C ABI of include/kohler.h). Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkohler.so")

OK, E_ARG, E_RANGE, E_CAPACITY, E_NOMEM, E_DEVICE, E_BUSY = 0, -1, -2, -3, -4, -5, -6
U8, U16 = 1, 2
MAX_M_U16 = 10200

# every symbol include/kohler.h declares
EXPORTS = (
    "kohler_create", "kohler_destroy", "kohler_strerror", "kohler_curve", "kohler_curve_async",
    "kohler_curve_batch", "kohler_set_plan", "kohler_get_plan",
)


class Plan(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("band", ctypes.c_int32), ("block", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("px_per_lane", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


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
    lib.kohler_set_plan.argtypes = [vp, ctypes.c_int, i32, i32, ctypes.POINTER(Plan)]
    lib.kohler_set_plan.restype = ctypes.c_int
    lib.kohler_get_plan.argtypes = [vp, ctypes.c_int, i64, i64, i32, i32, ctypes.POINTER(Plan)]
    lib.kohler_get_plan.restype = ctypes.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().kohler_strerror(status).decode()
