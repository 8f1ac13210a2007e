"""Roofline probes for the benchmark (``libkohler_roofline.so``, ``csrc/kohler_roofline.hip``).

``read_stream`` measures the HBM read rate of one pass over device buffers of the curve launch's
size (rotating over buffers that together exceed the 256 MB Infinity Cache), ``lds_atomics`` the
chip-wide rate of LDS atomic increments at several address patterns. Both time their launches with
HIP events on the stream they launch on. Not part of the curve library: the benchmark's reference
points only.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkohler_roofline.so")
PATTERNS = {"distinct": 0, "rand256": 1, "band_table": 2, "smooth_image": 3, "same_word": 4}
_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1707_05062_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
        lib.roof_read_stream.argtypes = [vp, u64, i32, i32, vp, vp]
        lib.roof_read_stream.restype = ctypes.c_int
        lib.roof_lds_atomics.argtypes = [i32, i32, i32, i32, vp, vp]
        lib.roof_lds_atomics.restype = ctypes.c_int
        lib.roof_lds_atomics_per_iter.argtypes = []
        lib.roof_lds_atomics_per_iter.restype = ctypes.c_int
        _lib = lib
    return _lib


def read_stream(torch, bufs, reps: int = 64, grid: int = 2048) -> dict:
    """Read rate (GB/s) of one launch reading one whole buffer, cycling over `bufs`: HIP events on
    the launch stream around `reps` back-to-back launches (as the curve kernel is timed), so that
    host launch latency stays out of the figure."""
    lib = load()
    dev = bufs[0].device
    sink = torch.zeros(64, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    nbytes = bufs[0].numel() * bufs[0].element_size()
    n16 = nbytes // 16 * 16
    for b in bufs[:4]:
        assert lib.roof_read_stream(b.data_ptr(), n16, grid, 256, sink.data_ptr(), stream.cuda_stream) == 0
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for i in range(reps):
        assert lib.roof_read_stream(bufs[(4 + i) % len(bufs)].data_ptr(), n16, grid, 256, sink.data_ptr(),
                                    stream.cuda_stream) == 0
    b.record(stream)
    torch.cuda.synchronize()
    t = a.elapsed_time(b) * 1e-3 / reps
    return {"bytes_per_launch": int(n16), "us_per_launch": t * 1e6, "gb_s": n16 / t / 1e9, "grid": grid,
            "block": 256, "launches": reps, "buffers": len(bufs)}


def lds_atomics(torch, num_cus: int, reps: int = 4, iters: int = 256, block: int = 1024,
                per_cu: int = 2) -> dict:
    """Chip-wide LDS atomic increments per second at each pattern: HIP events around `reps`
    back-to-back launches (after one warm-up launch), each workgroup's count checked."""
    lib = load()
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.current_stream(dev)
    grid = num_cus * per_cu
    outs = [torch.zeros(grid, dtype=torch.int32, device=dev) for _ in range(reps + 1)]
    per_iter = lib.roof_lds_atomics_per_iter()
    n = grid * block * iters * per_iter
    res = {"grid": grid, "block": block, "atomics_per_launch": n, "launches": reps}
    for name, pat in PATTERNS.items():
        for o in outs:
            o.zero_()
        assert lib.roof_lds_atomics(pat, iters, grid, block, outs[0].data_ptr(), stream.cuda_stream) == 0
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        for r in range(reps):
            assert lib.roof_lds_atomics(pat, iters, grid, block, outs[r + 1].data_ptr(), stream.cuda_stream) == 0
        b.record(stream)
        torch.cuda.synchronize()
        for o in outs:
            total = int(o.to(torch.int64).sum())
            assert total == n, f"LDS atomic probe {name}: counted {total}, expected {n}"
        res[name] = n * reps / (a.elapsed_time(b) * 1e-3)
    return res
