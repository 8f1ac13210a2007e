"""CPU oracle for the Köhler contrast curve (test infrastructure only).

Only the test suite, the smoke check and the bench's CPU-baseline leg may import this package. The
product path (the HIP library and its Python binding) never does, and it shares no code with it.

Reference: G. Noyel, arXiv 1707.05062. ``curve`` is the definition of Sec. 2.1 (eqs (1)-(3)) written
out over every threshold and every ordered neighbour pair; ``alg1`` is Algorithm 1 of Sec. 3.1 over
the half neighbourhood of Sec. 3.2; ``curve_nbhd`` and ``alg1_nbhd`` are the same two routes for
a symmetric structuring element or the hexagonal 6-neighbourhood; ``binomial3`` is a 3x3 low-pass
applied before the method (Sec. 5); ``thresholds`` gives the curve's local maxima and the optimum of
eq (4); ``segment`` labels pixels by the classes those thresholds cut (Sec. 2.1), ``class_stats`` and
``mean_image`` give each class's mean value, ``top_thresholds`` the most significant thresholds. The
C sources are in ``kohler_oracle.c``; ``build()`` compiles them with gcc and OpenMP.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kohler_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, E_ARG, E_RANGE, E_CAPACITY = 0, -1, -2, -3


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle into a shared library (plain gcc, -O2, OpenMP; no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           "-o", out, src]
    subprocess.run(cmd, check=True)
    return out


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(lib):
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.oracle_curve.argtypes = [i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                 i32p, ctypes.c_int32, i64p, i64p, f64p]
    lib.oracle_curve.restype = ctypes.c_int
    lib.oracle_alg1.argtypes = [i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                i64p, i64p]
    lib.oracle_alg1.restype = ctypes.c_int
    lib.oracle_thresholds.argtypes = [i64p, i64p, ctypes.c_int32, i32p, ctypes.c_int32, i32p, i32p]
    lib.oracle_thresholds.restype = ctypes.c_int
    lib.oracle_curve_nbhd.argtypes = [i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, i32p, i32p,
                                      ctypes.c_int32, ctypes.c_int32, i32p, ctypes.c_int32, i64p, i64p, f64p]
    lib.oracle_curve_nbhd.restype = ctypes.c_int
    lib.oracle_alg1_nbhd.argtypes = [i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, i32p, i32p,
                                     ctypes.c_int32, ctypes.c_int32, i64p, i64p]
    lib.oracle_alg1_nbhd.restype = ctypes.c_int
    return lib


def load_library(path: str):
    """Bind an oracle library built from another source file (used by the mutation tests)."""
    return _bind(ctypes.CDLL(path))


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def curve(img: np.ndarray, M: int, nbhd: int = 4, ts=None, lib=None):
    """Eqs (1)-(3) by enumeration: returns (sum int64, count int64, C float64) for t in ``ts``
    (all of 0..M-1 by default)."""
    lib = lib or _load()
    f = np.ascontiguousarray(img, dtype=np.int32)
    if f.ndim != 2:
        raise ValueError("image must be 2-D")
    t = np.arange(M, dtype=np.int32) if ts is None else np.ascontiguousarray(ts, dtype=np.int32)
    s = np.zeros(len(t), np.int64)
    k = np.zeros(len(t), np.int64)
    c = np.zeros(len(t), np.float64)
    st = lib.oracle_curve(_ptr(f, ctypes.c_int32), f.shape[0], f.shape[1], M, nbhd,
                          _ptr(t, ctypes.c_int32), len(t), _ptr(s, ctypes.c_int64),
                          _ptr(k, ctypes.c_int64), _ptr(c, ctypes.c_double))
    if st != OK:
        raise OracleError(st, "oracle_curve")
    return s, k, c


def alg1(img: np.ndarray, M: int, nbhd: int = 4, lib=None):
    """Algorithm 1 over the half neighbourhood: returns (sum int64, count int64)."""
    lib = lib or _load()
    f = np.ascontiguousarray(img, dtype=np.int32)
    s = np.zeros(M, np.int64)
    k = np.zeros(M, np.int64)
    st = lib.oracle_alg1(_ptr(f, ctypes.c_int32), f.shape[0], f.shape[1], M, nbhd,
                         _ptr(s, ctypes.c_int64), _ptr(k, ctypes.c_int64))
    if st != OK:
        raise OracleError(st, "oracle_alg1")
    return s, k


# ------------------------------------------------------------------------------------------------
# Other neighbourhoods (Sec. 2.1 names the 6-neighbourhood; Sec. 3.2's argument holds for any
# symmetric structuring element A and a half A* with one offset of each pair {a, -a}).

def full_of(half) -> list[tuple[int, int]]:
    """The symmetric set A = A* u -A* of a half set of (dy, dx) offsets."""
    out = []
    for dy, dx in half:
        out += [(int(dy), int(dx)), (-int(dy), -int(dx))]
    return out


def half_of(full_) -> list[tuple[int, int]]:
    """The canonical half of a symmetric set: the offsets with dy > 0, or dy == 0 and dx > 0."""
    return [(int(dy), int(dx)) for dy, dx in full_ if dy > 0 or (dy == 0 and dx > 0)]


def _offsets(offs):
    o = np.asarray(offs, dtype=np.int32).reshape(-1, 2) if offs is not None and len(offs) else np.zeros((0, 2), np.int32)
    return np.ascontiguousarray(o[:, 0]), np.ascontiguousarray(o[:, 1])


def curve_nbhd(img: np.ndarray, M: int, offsets=None, hex: bool = False, ts=None, lib=None):
    """Eqs (1)-(3) by enumeration over the full neighbourhood: the symmetric offset set `offsets`
    ((dy, dx) pairs, the same at every pixel), or with hex=True the 6-neighbourhood of a hexagonal
    grid stored with odd rows shifted right by half a pixel (see the C source). Returns (sum, count,
    C) for t in ``ts`` (all of 0..M-1 by default)."""
    lib = lib or _load()
    f = np.ascontiguousarray(img, dtype=np.int32)
    if f.ndim != 2:
        raise ValueError("image must be 2-D")
    dy, dx = _offsets(offsets)
    t = np.arange(M, dtype=np.int32) if ts is None else np.ascontiguousarray(ts, dtype=np.int32)
    s = np.zeros(len(t), np.int64)
    k = np.zeros(len(t), np.int64)
    c = np.zeros(len(t), np.float64)
    st = lib.oracle_curve_nbhd(_ptr(f, ctypes.c_int32), f.shape[0], f.shape[1], M, _ptr(dy, ctypes.c_int32),
                               _ptr(dx, ctypes.c_int32), len(dy), 1 if hex else 0, _ptr(t, ctypes.c_int32),
                               len(t), _ptr(s, ctypes.c_int64), _ptr(k, ctypes.c_int64), _ptr(c, ctypes.c_double))
    if st != OK:
        raise OracleError(st, "oracle_curve_nbhd")
    return s, k, c


def alg1_nbhd(img: np.ndarray, M: int, half=None, hex: bool = False, lib=None):
    """Algorithm 1 over a half neighbourhood (`half`: (dy, dx) offsets holding no offset with its
    negation; hex=True: the hexagonal grid's half). Returns (sum, count)."""
    lib = lib or _load()
    f = np.ascontiguousarray(img, dtype=np.int32)
    dy, dx = _offsets(half)
    s = np.zeros(M, np.int64)
    k = np.zeros(M, np.int64)
    st = lib.oracle_alg1_nbhd(_ptr(f, ctypes.c_int32), f.shape[0], f.shape[1], M, _ptr(dy, ctypes.c_int32),
                              _ptr(dx, ctypes.c_int32), len(dy), 1 if hex else 0, _ptr(s, ctypes.c_int64),
                              _ptr(k, ctypes.c_int64))
    if st != OK:
        raise OracleError(st, "oracle_alg1_nbhd")
    return s, k


# ------------------------------------------------------------------------------------------------
# A low-pass filter before the method (Sec. 5 suggests combining it with previous transforms; the
# paper names no filter, so this one is a reading: the 3x3 binomial kernel).

BINOMIAL3 = ((1, 2, 1), (2, 4, 2), (1, 2, 1))


def binomial3(img: np.ndarray) -> np.ndarray:
    """3x3 binomial low-pass: g(y, x) = floor((sum of w(i, j) f(y+i, x+j) over i, j in {-1, 0, 1}
    + 8) / 16) with the weights BINOMIAL3 (total 16), i.e. the weighted mean rounded half up;
    coordinates outside the image are replaced by the nearest pixel of the image (replicated
    borders). Values stay in [0, M) when f does. Same shape and dtype as the input."""
    a = np.asarray(img)
    f = a.astype(np.int64)
    H, W = f.shape
    acc = np.zeros((H, W), np.int64)
    for i in (-1, 0, 1):
        ys = np.clip(np.arange(H) + i, 0, H - 1)
        for j in (-1, 0, 1):
            xs = np.clip(np.arange(W) + j, 0, W - 1)
            acc += BINOMIAL3[i + 1][j + 1] * f[ys][:, xs]
    return ((acc + 8) // 16).astype(a.dtype)


def thresholds(sum_, count, cap: int | None = None, lib=None):
    """Local maxima (ascending) and t0 of eq (4) from exact int64 sums and counts.

    Returns (thresholds int32 array, t0, status); with a capacity below the number found the
    array is truncated and status is E_CAPACITY."""
    lib = lib or _load()
    s = np.ascontiguousarray(sum_, dtype=np.int64)
    k = np.ascontiguousarray(count, dtype=np.int64)
    M = len(s)
    cap = M if cap is None else cap
    thr = np.zeros(max(cap, 1), np.int32)
    n = ctypes.c_int32(0)
    t0 = ctypes.c_int32(0)
    st = lib.oracle_thresholds(_ptr(s, ctypes.c_int64), _ptr(k, ctypes.c_int64), M,
                               _ptr(thr, ctypes.c_int32), cap, ctypes.byref(n), ctypes.byref(t0))
    if st not in (OK, E_CAPACITY):
        raise OracleError(st, "oracle_thresholds")
    return thr[: min(n.value, cap)].copy(), int(t0.value), st, int(n.value)


def full(img: np.ndarray, M: int, nbhd: int = 4, lib=None):
    """Everything the hot path returns: (sum, count, C, thresholds, t0)."""
    s, k, c = curve(img, M, nbhd, lib=lib)
    thr, t0, _, _ = thresholds(s, k, lib=lib)
    return s, k, c, thr, t0


def segment(img: np.ndarray, thresholds_, rows_per_step: int = 256) -> np.ndarray:
    """Class label of every pixel for ascending thresholds t_1 < ... < t_k (Sec. 2.1): the lower set of
    threshold t is {f <= t} (eq (1)), so the thresholds cut the grey levels into k + 1 classes and a
    pixel of value f is in class #{i : t_i < f}. Written out as that count (a comparison with every
    threshold, summed), in row blocks to bound memory. Returns int32 labels of the image's shape."""
    f = np.asarray(img).astype(np.int64)
    t = np.asarray(thresholds_, dtype=np.int64).reshape(-1)
    out = np.zeros(f.shape, np.int32)
    if t.size == 0:
        return out
    f2 = f.reshape(f.shape[0], -1) if f.ndim > 1 else f.reshape(1, -1)
    o2 = out.reshape(f2.shape)
    for r in range(0, f2.shape[0], rows_per_step):
        blk = f2[r:r + rows_per_step]
        o2[r:r + rows_per_step] = (blk[..., None] > t[None, None, :]).sum(axis=-1)
    return out


def class_stats(img: np.ndarray, thresholds_, M: int):
    """Per-class pixel count, value sum and mean for the k + 1 classes that ascending thresholds cut
    (Sec. 2.1, where each class of Fig. 1 is shown at the mean value of its pixels; class of a pixel
    as in ``segment``). A value of M or more counts in class k with the
    value M. Written out class by class: count = number of pixels with that label, sum = their values
    added in int64, mean = sum / count as one float64 division (0.0 for an empty class). Returns
    (int64 count[k+1], int64 sum[k+1], float64 mean[k+1])."""
    f = np.minimum(np.asarray(img).astype(np.int64), M)
    lab = segment(f, thresholds_)
    k = len(np.asarray(thresholds_).reshape(-1))
    count = np.zeros(k + 1, np.int64)
    total = np.zeros(k + 1, np.int64)
    mean = np.zeros(k + 1, np.float64)
    for j in range(k + 1):
        sel = lab == j
        count[j] = int(sel.sum())
        total[j] = int(f[sel].sum(dtype=np.int64))
        if count[j]:
            mean[j] = np.float64(total[j]) / np.float64(count[j])
    return count, total, mean


def mean_image(img: np.ndarray, thresholds_, M: int) -> np.ndarray:
    """Every pixel replaced by the mean of its class (``class_stats``), rounded to the nearest
    integer with ties to even, in the image's own dtype."""
    img = np.asarray(img)
    _, _, mean = class_stats(img, thresholds_, M)
    lab = segment(np.minimum(img.astype(np.int64), M), thresholds_)
    return np.rint(mean)[lab].astype(img.dtype)


def top_thresholds(sum_, count, thresholds_, k: int):
    """The k most significant thresholds (Sec. 2.1, the discussion of Fig. 1; the paper does not define
    "most significant", so this takes the reading: largest contrast first): the thresholds ordered by C(t) = sum(t) / count(t)
    descending (0 where count is 0), compared as exact rationals, equal C in ascending t; the first
    min(k, n) of that order."""
    from fractions import Fraction

    def key(t):
        c = int(count[t])
        return (-(Fraction(int(sum_[t]), c) if c else Fraction(0)), int(t))

    return [int(t) for t in sorted((int(t) for t in thresholds_), key=key)[:max(0, k)]]
