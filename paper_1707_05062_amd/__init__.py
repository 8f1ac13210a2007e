"""Köhler contrast-thresholding curve on MI355X (gfx950).

Python binding over the C ABI of ``include/kohler.h`` (``libkohler.so``). Every step of the curve
runs in the library's HIP kernels; this module only marshals arguments. PyTorch supplies device
memory and streams.

Reference: G. Noyel, "Speeding up the Köhler's method of contrast thresholding", arXiv 1707.05062.
For every integer threshold t the library returns the exact sum of the pair contrasts over the
boundary B(t) (Sec. 2.1, eqs (1)-(2)), #B(t), the mean contrast C(t) (eq (3)), the local maxima of
C (the multiple thresholds) and the optimum t0 (eq (4)).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import (E_ARG, E_BUSY, E_CANCELED, E_CAPACITY, E_DEVICE, E_NOMEM, E_RANGE, OK,  # noqa: F401
                   Plan, RequestInfo, ServerConfig, ServerCounters)

__all__ = ["Context", "CurveResult", "KohlerError", "Plan", "Server", "curve", "curve_noalloc",
           "default_context", "strerror"]

FORM_AUTO, FORM_BAND, FORM_MARG, FORM_TRI = 0, 1, 2, 3


class KohlerError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        super().__init__(f"{what}: {_lib.strerror(status)} ({status})" if what else _lib.strerror(status))
        self.status = status


def strerror(status: int) -> str:
    return _lib.strerror(status)


@dataclass
class CurveResult:
    sum: object         # int64[M]
    count: object       # int64[M]
    C: object           # float64[M]
    thresholds: object  # int32[n] (truncated to the capacity)
    t0: int
    n_thresholds: int
    status: int


def _torch():
    import torch
    return torch


def _dtype_code(dt) -> int:
    torch = _torch()
    if dt in (torch.uint8, np.uint8):
        return _lib.U8
    if dt in (getattr(torch, "uint16", None), np.uint16):
        return _lib.U16
    raise TypeError(f"unsupported pixel dtype {dt}; use uint8 or uint16")


def _image_args(img):
    """(pointer, dtype code, H, W, pitch, keepalive) for a 2-D torch tensor or numpy array."""
    torch = _torch()
    if isinstance(img, torch.Tensor):
        if img.dim() != 2 or img.stride(1) != 1:
            raise ValueError("image must be a 2-D tensor with unit column stride")
        H, W = img.shape
        pitch = img.stride(0) if H > 1 else W
        return img.data_ptr(), _dtype_code(img.dtype), int(H), int(W), int(pitch), img
    a = np.asarray(img)
    if a.ndim != 2:
        raise ValueError("image must be 2-D")
    if a.dtype not in (np.uint8, np.uint16):
        raise TypeError("numpy images must be uint8 or uint16")
    a = np.ascontiguousarray(a)
    H, W = a.shape
    return a.ctypes.data, _dtype_code(a.dtype.type), int(H), int(W), int(W), a


def _label_args(buf):
    """(pointer, H, W, pitch, keepalive) of a writable 2-D uint8 destination with unit column stride:
    a torch tensor (host, pinned or device) or a numpy array, used in place (never copied)."""
    torch = _torch()
    if isinstance(buf, torch.Tensor):
        if buf.dim() != 2 or buf.stride(1) != 1 or buf.dtype != torch.uint8:
            raise ValueError("labels must be a 2-D uint8 tensor with unit column stride")
        H, W = buf.shape
        return buf.data_ptr(), int(H), int(W), int(buf.stride(0) if H > 1 else W), buf
    a = buf
    if not isinstance(a, np.ndarray) or a.ndim != 2 or a.dtype != np.uint8 or a.strides[1] != 1 or not a.flags.writeable:
        raise ValueError("labels must be a writable 2-D uint8 array with unit column stride")
    H, W = a.shape
    return a.ctypes.data, int(H), int(W), int(a.strides[0] if H > 1 else W), a


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _complete(img):
    """Entry points that work on the library's own streams (the synchronous curve, the autotuner,
    server submission) read a device image without waiting for the caller's streams: wait here for
    torch's current stream of the image's device, which produced it in the usual case."""
    torch = _torch()
    if isinstance(img, torch.Tensor) and img.is_cuda:
        torch.cuda.current_stream(img.device).synchronize()


class Context:
    """A library context bound to one HIP device (owns device scratch and a stream)."""

    def __init__(self, device: int = 0, lib_path: str | None = None):
        # lib_path: another build of the same library (e.g. the phase-clock measurement build)
        self._lib = _lib.load() if lib_path is None else _lib.load(lib_path)
        self._h = ctypes.c_void_p()
        st = self._lib.kohler_create(ctypes.byref(self._h), int(device))
        if st != OK:
            raise KohlerError(st, "kohler_create")
        self.device = int(device)

    def close(self):
        if self._h:
            self._lib.kohler_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- plans -------------------------------------------------------------------------------
    def set_plan(self, dtype: int, M: int, nbhd: int, form: int = FORM_AUTO, band: int = 0,
                 block: int = 512, grid: int = 0, px_per_lane: int = 4, replicas: int = 0, copies: int = 0,
                 acc_split: int = 0):
        pl = Plan(form, band, block, grid, px_per_lane, replicas, copies, acc_split)
        st = self._lib.kohler_set_plan(self._h, dtype, M, nbhd, ctypes.byref(pl))
        if st != OK:
            raise KohlerError(st, "kohler_set_plan")

    def get_plan(self, dtype: int, H: int, W: int, M: int, nbhd: int) -> dict:
        pl = Plan()
        st = self._lib.kohler_get_plan(self._h, dtype, H, W, M, nbhd, ctypes.byref(pl))
        if st != OK:
            raise KohlerError(st, "kohler_get_plan")
        return pl.as_dict()

    def autotune(self, imgs, M: int, nbhd: int = 4, reps: int = 5) -> tuple[dict, float]:
        """Run the library's autotuner on device images (one image tunes the single-image launch,
        several the batched one); the chosen plan is stored in this context. Returns (plan, us)."""
        torch = _torch()
        imgs = list(imgs)
        n = len(imgs)
        ptrs = (ctypes.c_void_p * n)()
        Hs, Ws, Ps = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
        code = None
        for i, im in enumerate(imgs):
            if not isinstance(im, torch.Tensor) or not im.is_cuda:
                raise ValueError("autotune takes device tensors")
            p, c, H, W, pitch, _ = _image_args(im)
            if code is not None and c != code:
                raise TypeError("all images must share one dtype")
            code = c
            ptrs[i], Hs[i], Ws[i], Ps[i] = p, H, W, pitch
            _complete(im)
        best = Plan()
        us = ctypes.c_double(0.0)
        st = self._lib.kohler_autotune(self._h, n, ptrs, Hs, Ws, Ps, code, M, nbhd, reps,
                                       ctypes.byref(best), ctypes.byref(us))
        if st != OK:
            raise KohlerError(st, "kohler_autotune")
        return best.as_dict(), float(us.value)

    # -- segmentation ------------------------------------------------------------------------
    def segment(self, img, thr, n_thr, capacity: int, M: int, out=None, label_dtype=None, stream=None):
        """Enqueue the class labels of a device image for device thresholds `thr` (int32) and the
        device count `n_thr` (an int32 tensor element, e.g. a curve call's ints[0:1]): label =
        number of thresholds below the pixel value. Returns the label tensor (uint8 when the
        capacity is at most 255, else uint16, unless label_dtype says otherwise)."""
        torch = _torch()
        ptr, code, H, W, pitch, keep = _image_args(img)
        if label_dtype is None:
            label_dtype = torch.uint8 if capacity <= 255 else torch.uint16
        lcode = _lib.U8 if label_dtype == torch.uint8 else _lib.U16
        if out is None:
            out = torch.empty((H, W), dtype=label_dtype, device=torch.device("cuda", self.device))
        if out.dim() != 2 or out.stride(1) != 1 or tuple(out.shape) != (H, W):
            raise ValueError("labels must be an H x W tensor with unit column stride")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        st = self._lib.kohler_segment(self._h, ctypes.c_void_p(ptr), code, H, W, pitch, M, _ptr(thr),
                                      ctypes.c_void_p(n_thr.data_ptr()), int(capacity), _ptr(out), lcode,
                                      out.stride(0) if H > 1 else W, ctypes.c_void_p(s.cuda_stream))
        del keep
        if st != OK:
            raise KohlerError(st, "kohler_segment")
        return out

    def class_stats(self, img, thr, n_thr, capacity: int, M: int, stream=None):
        """Enqueue the per-class pixel count, value sum and mean (device tensors of capacity + 1
        entries: int64, int64, float64) of a device image for the device thresholds `thr` and count
        `n_thr`, classes as in `segment`."""
        torch = _torch()
        ptr, code, H, W, pitch, keep = _image_args(img)
        dev = torch.device("cuda", self.device)
        count = torch.empty(capacity + 1, dtype=torch.int64, device=dev)
        total = torch.empty(capacity + 1, dtype=torch.int64, device=dev)
        mean = torch.empty(capacity + 1, dtype=torch.float64, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        st = self._lib.kohler_class_stats(self._h, ctypes.c_void_p(ptr), code, H, W, pitch, M, _ptr(thr),
                                          ctypes.c_void_p(n_thr.data_ptr()), int(capacity), _ptr(count),
                                          _ptr(total), _ptr(mean), ctypes.c_void_p(s.cuda_stream))
        del keep
        if st != OK:
            raise KohlerError(st, "kohler_class_stats")
        return count, total, mean

    def mean_image(self, img, thr, n_thr, capacity: int, M: int, mean, out=None, stream=None):
        """Enqueue the class-mean image (each pixel replaced by its class's mean rounded to nearest,
        ties to even, in the image's dtype) for class means `mean` (float64 device tensor)."""
        torch = _torch()
        ptr, code, H, W, pitch, keep = _image_args(img)
        if out is None:
            out = torch.empty((H, W), dtype=img.dtype, device=torch.device("cuda", self.device))
        if out.dim() != 2 or out.stride(1) != 1 or tuple(out.shape) != (H, W) or out.dtype != img.dtype:
            raise ValueError("the output must be an H x W tensor of the image's dtype with unit column stride")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        st = self._lib.kohler_mean_image(self._h, ctypes.c_void_p(ptr), code, H, W, pitch, M, _ptr(thr),
                                         ctypes.c_void_p(n_thr.data_ptr()), int(capacity), _ptr(mean), _ptr(out),
                                         out.stride(0) if H > 1 else W, ctypes.c_void_p(s.cuda_stream))
        del keep
        if st != OK:
            raise KohlerError(st, "kohler_mean_image")
        return out

    def top_thresholds(self, sum_, count, thr, n_thr, capacity: int, M: int, k: int, stream=None):
        """Enqueue the k most significant thresholds (largest C first, equal C in ascending t) of a
        device curve (`sum_`, `count`: int64[M]) and its device thresholds. Returns (top int32[k],
        n_top int32[1]) device tensors."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        top = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
        n_top = torch.empty(1, dtype=torch.int32, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        st = self._lib.kohler_top_thresholds(self._h, _ptr(sum_), _ptr(count), M, _ptr(thr),
                                             ctypes.c_void_p(n_thr.data_ptr()), int(capacity), int(k), _ptr(top),
                                             _ptr(n_top), ctypes.c_void_p(s.cuda_stream))
        if st != OK:
            raise KohlerError(st, "kohler_top_thresholds")
        return top, n_top

    # -- synchronous -------------------------------------------------------------------------
    def curve(self, img, M: int, nbhd: int = 4, capacity: int | None = None,
              check: bool = True) -> CurveResult:
        """Curve of one image (device tensor or host array); results as numpy arrays."""
        ptr, code, H, W, pitch, keep = _image_args(img)
        _complete(img)
        cap = M if capacity is None else int(capacity)
        m = max(int(M), 1)  # the library validates M; the buffers only need to exist
        s = np.zeros(m, np.int64)
        k = np.zeros(m, np.int64)
        c = np.zeros(m, np.float64)
        thr = np.zeros(max(cap, 1), np.int32)
        n = ctypes.c_int32(0)
        t0 = ctypes.c_int32(0)
        i64p, i32p = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
        st = self._lib.kohler_curve(
            self._h, ctypes.c_void_p(ptr), code, H, W, pitch, M, nbhd,
            s.ctypes.data_as(i64p), k.ctypes.data_as(i64p),
            c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), thr.ctypes.data_as(i32p), cap,
            ctypes.byref(n), ctypes.byref(t0))
        del keep
        if check and st not in (OK, E_CAPACITY):
            raise KohlerError(st, "kohler_curve")
        return CurveResult(s, k, c, thr[: min(n.value, cap)].copy(), int(t0.value), int(n.value), st)

    # -- stream-ordered ----------------------------------------------------------------------
    def alloc_outputs(self, M: int, capacity: int, n: int | None = None):
        """Device output tensors for curve_async (n=None) or curve_batch (n images)."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        shape = (M,) if n is None else (n, M)
        m = 1 if n is None else n
        return dict(
            sum=torch.zeros(shape, dtype=torch.int64, device=dev),
            count=torch.zeros(shape, dtype=torch.int64, device=dev),
            C=torch.zeros(shape, dtype=torch.float64, device=dev),
            thr=torch.zeros((max(capacity, 1),) if n is None else (n, max(capacity, 1)),
                            dtype=torch.int32, device=dev),
            ints=torch.zeros((3 * m,), dtype=torch.int32, device=dev),
        )

    def curve_async(self, img, M: int, nbhd: int = 4, capacity: int | None = None, out=None,
                    stream=None):
        """Enqueue the curve of a device image on `stream` (torch's current stream by default).
        Returns the output dict: sum, count, C, thr (device tensors) and ints = [n_thr, t0, status]."""
        torch = _torch()
        ptr, code, H, W, pitch, keep = _image_args(img)
        cap = M if capacity is None else int(capacity)
        out = out or self.alloc_outputs(M, cap)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        ints = out["ints"]
        base = ints.data_ptr()
        st = self._lib.kohler_curve_async(
            self._h, ctypes.c_void_p(ptr), code, H, W, pitch, M, nbhd, _ptr(out["sum"]),
            _ptr(out["count"]), _ptr(out["C"]), _ptr(out["thr"]), cap, ctypes.c_void_p(base),
            ctypes.c_void_p(base + 4), ctypes.c_void_p(base + 8), ctypes.c_void_p(s.cuda_stream))
        del keep
        if st != OK:
            raise KohlerError(st, "kohler_curve_async")
        return out

    def curve_nbhd_async(self, img, M: int, half=None, hex: bool = False, prefilter: bool = False,
                         capacity: int | None = None, out=None, stream=None):
        """Enqueue the curve of a device image for another neighbourhood: the symmetric structuring
        element with half offsets `half` ((dy, dx) pairs), or hex=True for the hexagonal grid (odd
        rows shifted right by half a pixel); prefilter=True takes the curve of the 3x3 binomial
        low-pass of the image. Outputs as curve_async."""
        torch = _torch()
        ptr, code, H, W, pitch, keep = _image_args(img)
        cap = M if capacity is None else int(capacity)
        out = out or self.alloc_outputs(M, cap)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        nb = _lib.Nbhd()
        if hex:
            nb.kind = _lib.NBHD_HEX6
        else:
            offs = [(int(dy), int(dx)) for dy, dx in (half or [])]
            if len(offs) > _lib.NBHD_MAX_HALF:
                raise ValueError(f"at most {_lib.NBHD_MAX_HALF} half offsets")
            nb.kind = _lib.NBHD_OFFSETS
            nb.n_half = len(offs)
            for i, (dy, dx) in enumerate(offs):
                nb.half_dy[i], nb.half_dx[i] = dy, dx
        ints = out["ints"]
        base = ints.data_ptr()
        st = self._lib.kohler_curve_nbhd_async(
            self._h, ctypes.c_void_p(ptr), code, H, W, pitch, M, ctypes.byref(nb), 1 if prefilter else 0,
            _ptr(out["sum"]), _ptr(out["count"]), _ptr(out["C"]), _ptr(out["thr"]), cap, ctypes.c_void_p(base),
            ctypes.c_void_p(base + 4), ctypes.c_void_p(base + 8), ctypes.c_void_p(s.cuda_stream))
        del keep
        if st != OK:
            raise KohlerError(st, "kohler_curve_nbhd_async")
        return out

    def curve_nbhd(self, img, M: int, half=None, hex: bool = False, prefilter: bool = False,
                   capacity: int | None = None, check: bool = True) -> CurveResult:
        """curve_nbhd_async on torch's current stream, waited for; results as numpy arrays."""
        torch = _torch()
        out = self.curve_nbhd_async(img, M, half=half, hex=hex, prefilter=prefilter, capacity=capacity)
        torch.cuda.current_stream(self.device).synchronize()
        n, t0, st = [int(x) for x in out["ints"].cpu()]
        if check and st not in (OK, E_CAPACITY):
            raise KohlerError(st, "kohler_curve_nbhd_async")
        cap = M if capacity is None else int(capacity)
        return CurveResult(out["sum"].cpu().numpy(), out["count"].cpu().numpy(), out["C"].cpu().numpy(),
                           out["thr"].cpu().numpy()[: min(n, cap)].copy(), t0, n, st)

    def curve_batch(self, imgs, M: int, nbhd: int = 4, capacity: int | None = None, out=None,
                    stream=None):
        """Enqueue the curves of n device images (one persistent launch). Outputs are [n, M] etc.;
        ints is [n_thr(n), t0(n), status(n)] concatenated."""
        torch = _torch()
        n = len(imgs)
        cap = M if capacity is None else int(capacity)
        out = out or self.alloc_outputs(M, cap, n)
        ptrs = (ctypes.c_void_p * n)()
        Hs = (ctypes.c_int64 * n)()
        Ws = (ctypes.c_int64 * n)()
        Ps = (ctypes.c_int64 * n)()
        code = None
        for i, im in enumerate(imgs):
            p, c, H, W, pitch, _ = _image_args(im)
            if not isinstance(im, torch.Tensor) or not im.is_cuda:
                raise ValueError("curve_batch takes device tensors")
            if code is not None and c != code:
                raise TypeError("all images of a batch must share one dtype")
            code = c
            ptrs[i], Hs[i], Ws[i], Ps[i] = p, H, W, pitch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        ints = out["ints"]
        base = ints.data_ptr()
        st = self._lib.kohler_curve_batch(
            self._h, n, ptrs, Hs, Ws, Ps, code, M, nbhd, _ptr(out["sum"]), _ptr(out["count"]),
            _ptr(out["C"]), _ptr(out["thr"]), cap, ctypes.c_void_p(base),
            ctypes.c_void_p(base + 4 * n), ctypes.c_void_p(base + 8 * n),
            ctypes.c_void_p(s.cuda_stream))
        if st != OK:
            raise KohlerError(st, "kohler_curve_batch")
        return out


class Server:
    """A serving loop on a context's device (kohler_server_*): submit images as they arrive,
    collect results by ticket. See include/kohler.h for admission and batching."""

    def __init__(self, ctx: Context, dtype: int = _lib.U8, M: int = 256, nbhd: int = 4,
                 slots: int = 16, lanes: int = 2, max_batch: int = 16, queue_capacity: int = 4096,
                 thr_capacity: int | None = None, use_graphs: bool = False,
                 hbm_budget_bytes: int = 1 << 30, label_t0: bool = False):
        self._lib = _lib.load()
        self.ctx = ctx  # the context must outlive the server
        self.M = int(M)
        self.thr_capacity = self.M if thr_capacity is None else int(thr_capacity)
        self.dtype = int(dtype)
        cfg = ServerConfig(int(dtype), int(M), int(nbhd), int(slots), int(lanes), int(max_batch),
                           int(queue_capacity), self.thr_capacity, 1 if use_graphs else 0,
                           1 if label_t0 else 0, int(hbm_budget_bytes))
        self._h = ctypes.c_void_p()
        st = self._lib.kohler_server_create(ctx._h, ctypes.byref(cfg), ctypes.byref(self._h))
        if st != OK:
            raise KohlerError(st, "kohler_server_create")
        self._keep: dict[int, object] = {}

    def close(self):
        if self._h:
            self._lib.kohler_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, img, labels=None) -> int:
        """Queue one image (host array, pinned tensor or device tensor); returns its ticket.
        Video mode (label_t0=True): `labels`, a uint8 H x W array or tensor (host, pinned or device)
        with unit column stride, receives the image's two-class segmentation at its own t0 by the
        time wait() returns. Raises KohlerError(E_BUSY) when admission is refused."""
        ptr, code, H, W, pitch, keep = _image_args(img)
        if code != self.dtype:
            raise TypeError("image dtype does not match the server")
        _complete(img)
        t = ctypes.c_uint64(0)
        if labels is None:
            st = self._lib.kohler_server_submit(self._h, ctypes.c_void_p(ptr), H, W, pitch, ctypes.byref(t))
        else:
            lptr, lH, lW, lpitch, lkeep = _label_args(labels)
            if (lH, lW) != (H, W):
                raise ValueError("labels must have the image's shape")
            _complete(labels)
            keep = (keep, lkeep)
            st = self._lib.kohler_server_submit_labels(self._h, ctypes.c_void_p(ptr), H, W, pitch,
                                                       ctypes.c_void_p(lptr), lpitch, ctypes.byref(t))
        if st != OK:
            raise KohlerError(st, "kohler_server_submit")
        self._keep[t.value] = keep  # the image (and labels) must stay alive until the request completes
        return int(t.value)

    def poll(self, ticket: int) -> bool:
        st = self._lib.kohler_server_poll(self._h, ticket)
        if st < 0:
            raise KohlerError(st, "kohler_server_poll")
        return st == 1

    def wait(self, ticket: int) -> tuple[CurveResult, dict]:
        """Block until the request is done; returns its CurveResult and its info (status,
        n_thresholds, t0, batch, graph, t_submit_ns, t_launch_ns, t_done_ns)."""
        M, cap = self.M, self.thr_capacity
        s = np.zeros(M, np.int64)
        k = np.zeros(M, np.int64)
        c = np.zeros(M, np.float64)
        thr = np.zeros(max(cap, 1), np.int32)
        info = RequestInfo()
        st = self._lib.kohler_server_wait(self._h, ticket, s.ctypes.data, k.ctypes.data, c.ctypes.data,
                                          thr.ctypes.data, cap, ctypes.byref(info))
        self._keep.pop(ticket, None)
        if st == E_ARG:
            raise KohlerError(st, "kohler_server_wait")
        n = int(info.n_thresholds)
        return CurveResult(s, k, c, thr[: max(0, min(n, cap))].copy(), int(info.t0), n, st), info.as_dict()

    def cancel(self, ticket: int) -> bool:
        """True if the request was still queued and is now cancelled."""
        st = self._lib.kohler_server_cancel(self._h, ticket)
        if st == E_ARG:
            raise KohlerError(st, "kohler_server_cancel")
        return st == OK

    def pause(self, paused: bool = True):
        self._lib.kohler_server_pause(self._h, 1 if paused else 0)

    def stats(self) -> dict:
        out = ServerCounters()
        st = self._lib.kohler_server_stats(self._h, ctypes.byref(out))
        if st != OK:
            raise KohlerError(st, "kohler_server_stats")
        return out.as_dict()


_default: dict[int, Context] = {}


def default_context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def curve(img, M: int, nbhd: int = 4, capacity: int | None = None) -> CurveResult:
    """Synchronous curve of one image on the default context of device 0."""
    return default_context(0).curve(img, M, nbhd, capacity)


def curve_noalloc(img, M: int, nbhd: int = 4, capacity: int | None = None, out=None, stream=None,
                  plan: dict | None = None):
    """Enqueue the curve of a device image through kohler_curve_noalloc, the entry point that
    allocates nothing (its scratch is the library's per-GPU device array). `out` is a dict as
    Context.alloc_outputs returns it (the caller allocates outputs beforehand when it cannot
    allocate later); `plan` a dict of kohler_plan fields or None for the default plan."""
    torch = _torch()
    lib = _lib.load()
    ptr, code, H, W, pitch, keep = _image_args(img)
    cap = M if capacity is None else int(capacity)
    if out is None:
        dev = torch.device("cuda", torch.cuda.current_device())
        out = dict(sum=torch.zeros(M, dtype=torch.int64, device=dev), count=torch.zeros(M, dtype=torch.int64, device=dev),
                   C=torch.zeros(M, dtype=torch.float64, device=dev),
                   thr=torch.zeros(max(cap, 1), dtype=torch.int32, device=dev),
                   ints=torch.zeros(3, dtype=torch.int32, device=dev))
    s = stream if stream is not None else torch.cuda.current_stream()
    pl = None if plan is None else ctypes.byref(Plan(*[int(plan.get(k, 0)) for k, _ in Plan._fields_]))
    base = out["ints"].data_ptr()
    st = lib.kohler_curve_noalloc(ctypes.c_void_p(ptr), code, H, W, pitch, M, nbhd, _ptr(out["sum"]),
                                  _ptr(out["count"]), _ptr(out["C"]), _ptr(out["thr"]), cap,
                                  ctypes.c_void_p(base), ctypes.c_void_p(base + 4), ctypes.c_void_p(base + 8),
                                  pl, ctypes.c_void_p(s.cuda_stream))
    del keep
    if st != OK:
        raise KohlerError(st, "kohler_curve_noalloc")
    return out
