#!/usr/bin/env python3
"""Benchmark of the Köhler contrast curve on one MI355X.

Headline (one "step" = the whole hot path for one image: pair formation, per-pair accumulation,
merge, prefix sums, FP64 division, local maxima and t0, all in one launch):
  a 3456x5184 (about 18 MP) uint8 synthetic image, M = 256, 4-neighbourhood.
The image is resident in HBM before the timed region; the timed steps rotate over --rotate distinct
copies (32 x 17.9 MB = 573 MB) so that the 256 MB Infinity Cache cannot serve them. The launch plan
comes from the library's autotuner, run on the image before timing (or from --plan).

Also measured in the same run (reported beside the headline, not as separate lines):
  segment  the labels of the same image by its thresholds (a read-once, write-once stream);
  batched  96 uint8 images of log-uniform sizes (128^2 .. 4000x3000) in one persistent launch vs the
           plain kernel launched once per image on one stream;
  served   a Poisson stream of 240 requests/s (70% 1080p video frames, 20% 4K frames, 10% 18 MP
           stills) through the serving loop (eager launches, the default; with per-shape HIP graphs;
           and in video mode, where each request also gets its two-class labels at its own t0) vs
           the same loop restricted to one image per launch, with p50/p99 latency from scheduled
           arrival to results (and labels) in host memory, plus a burst that saturates them.
  other    the 256x256 and 4096^2 12-bit (N4, N8) workloads, the hexagonal 6-neighbourhood and the
           pre-filtered N4 curve of the 18 MP image.

Prints ONE JSON line with the headline throughput in Gpixel/s, the roofline of the curve kernel
(algorithmic bytes / average kernel duration from HIP events on the launch stream) and the CPU
oracle's throughput on the host cores (the CPU baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import queue
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E datasheet peak
METRIC = "Gpixel/s for Köhler C(t) curve (18MP, M=256) + % HBM roofline; p50/p99 frame ms"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


# ------------------------------------------------------------------------------------------------
# CPU baseline: the oracle as it stands

def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


ONE_THREAD_SNIPPET = """
import sys, time, numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
img = np.load(sys.argv[2])
oracle.curve(img[:8], int(sys.argv[3]), int(sys.argv[4]))
t = time.perf_counter()
oracle.curve(img, int(sys.argv[3]), int(sys.argv[4]))
print(time.perf_counter() - t)
"""


def cpu_baseline(img: np.ndarray, M: int, nbhd: int, runs: int = 3, one_thread_rows: int = 864) -> dict:
    """The oracle (plain brute force of eqs (1)-(3), OpenMP over thresholds) on the host cores, and
    on one core (in a child process started with OMP_NUM_THREADS=1) over the first rows."""
    import subprocess
    import tempfile

    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    times = []
    for _ in range(runs):
        t = time.perf_counter()
        oracle.curve(img, M, nbhd)
        times.append(time.perf_counter() - t)
    dt = float(np.median(times))
    res = {"value": img.size / dt / 1e9, "unit": "Gpixel/s", "cores": cores, "kind": "oracle",
           "seconds": dt, "cpu_model": cpu_model(),
           "sample": f"the full {img.shape[0]}x{img.shape[1]} image, all {M} thresholds, "
                     f"median of {runs} runs"}
    part = np.ascontiguousarray(img[:one_thread_rows])
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "rows.npy")
        np.save(path, part)
        env = dict(os.environ, OMP_NUM_THREADS="1")
        out = subprocess.run([sys.executable, "-c", ONE_THREAD_SNIPPET, ROOT, path, str(M), str(nbhd)],
                             env=env, capture_output=True, text=True, timeout=600)
    if out.returncode == 0:
        t1 = float(out.stdout.strip().splitlines()[-1])
        res["one_thread"] = {"value": part.size / t1 / 1e9, "unit": "Gpixel/s", "cores": 1, "seconds": t1,
                             "sample": f"the first {part.shape[0]} rows ({part.shape[0]}x{part.shape[1]}), "
                                       f"all {M} thresholds, one run"}
    else:
        res["one_thread"] = {"error": out.stderr.strip()[-300:]}
    return res


# ------------------------------------------------------------------------------------------------
# headline: one 18 MP image per launch

TRAFFIC_FILE = os.path.join(ROOT, "paper_1707_05062_amd", "traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1707_05062_amd", "csrc", f)
                  for f in ("kohler_kernels.hip", "kohler_impl.h")]


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(plan: dict):
    """HBM bytes per launch from the stored FETCH_SIZE/WRITE_SIZE measurements, if one was taken on
    this kernel build with the same strip width and grid (the other plan fields do not change the
    memory traffic of a launch beyond a few KB); else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256") != kernel_sources_digest():
        return None
    for row in t.get("by_tile_and_grid", []):
        if row["px_per_lane"] == plan.get("px_per_lane") and row["grid"] == plan.get("grid"):
            return {"bytes": row["traffic_bytes_per_launch"],
                    "source": f"{t['method']}; measured with plan {row['plan']}"}
    return None


def latency_ms(durs) -> dict:
    d = np.asarray(durs) * 1e3
    return {"n": int(len(d)), "mean": float(d.mean()), "p10": pct(d, 10), "p50": pct(d, 50), "p90": pct(d, 90),
            "p99": pct(d, 99)}


def lds_atomic_roofline(plan: dict, pairs: int, npx: int, kern_s: float, probe: dict) -> dict:
    """LDS atomics per launch by the plan's form: one per pair for the joint histograms (banded,
    triangular), two per pair plus one per pixel for the marginal histograms; the large-gap pass
    of the banded form (two more per pair of gap > band) is not counted. Peak: the probe's
    distinct-address rate (no two lanes of an instruction on one bank)."""
    per_launch = (2 * pairs + npx) if plan.get("form") == 2 else pairs
    achieved = per_launch / kern_s
    return {"achieved": achieved, "peak": probe["distinct"], "unit": "atomics/s",
            "frac": achieved / probe["distinct"], "atomics_per_launch": per_launch,
            "probe": {k: probe[k] for k in ("distinct", "rand256", "band_table", "smooth_image", "same_word")},
            "probe_launch": {"grid": probe["grid"], "block": probe["block"],
                             "atomics_per_launch": probe["atomics_per_launch"]}}


def parse_plan(s: str) -> dict:
    keys = ("form", "band", "block", "grid", "px_per_lane", "replicas", "copies")
    vals = [int(x) for x in s.split(":")]
    return dict(zip(keys, vals))


def headline(args, K, ctx, torch, gen) -> tuple[dict, np.ndarray]:
    from paper_1707_05062_amd import _lib
    cfg = gen.CONFIGS["cfg2"]
    H, W, M, nbhd = cfg["H"], cfg["W"], cfg["M"], 4
    img = gen.cfg2_image()
    log(f"cfg2 generated {img.shape}")
    dev = torch.device("cuda", 0)
    src = torch.from_numpy(img).to(dev)
    bufs = [src.clone() for _ in range(max(1, args.rotate))]
    if args.plan:
        ctx.set_plan(_lib.U8, M, nbhd, **parse_plan(args.plan))
        tuned = {"source": "--plan"}
    else:
        plan, us = ctx.autotune([bufs[0]], M, nbhd, reps=15)  # medians of 15 launches: a steadier pick
        tuned = {"source": "autotuner", "plan": plan, "median_us": us}
        log(f"autotuned plan {plan} {us:.2f} us")
    outs = ctx.alloc_outputs(M, M)
    stream = torch.cuda.current_stream(dev)

    # self-check on the first buffer: closed-form totals over the curve (sum_t #B(t) = sum of gaps)
    ctx.curve_async(bufs[0], M, nbhd, out=outs)
    torch.cuda.synchronize()
    f = img.astype(np.int64)
    gaps = np.concatenate([np.abs(f[:, 1:] - f[:, :-1]).ravel(), np.abs(f[1:] - f[:-1]).ravel()])
    cnt = outs["count"].cpu().numpy()
    sm = outs["sum"].cpu().numpy()
    n_thr, t0, status = [int(x) for x in outs["ints"].cpu()]
    selfcheck = bool(cnt.sum() == gaps.sum() and sm.sum() == (gaps * gaps // 4).sum() and status == 0)
    plan_used = ctx.get_plan(_lib.U8, H, W, M, nbhd)
    log(f"selfcheck={selfcheck} thresholds={n_thr} t0={t0} plan={plan_used}")

    for i in range(args.warmup):
        ctx.curve_async(bufs[i % len(bufs)], M, nbhd, out=outs)
    torch.cuda.synchronize()

    # timed region: back-to-back launches, HIP events on the launch stream around all of them
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):  # continue the rotation: the least recently used buffer first
        ctx.curve_async(bufs[(args.warmup + i) % len(bufs)], M, nbhd, out=outs, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_begin
    kern = ev0.elapsed_time(ev1) * 1e-3 / args.steps  # seconds per launch

    # frame latency: each launch bracketed by its own events (dispatch to completion), at least 100
    nlat = max(100, min(args.steps, 1000))
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(nlat)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(nlat)]
    for i in range(nlat):
        starts[i].record(stream)
        ctx.curve_async(bufs[(args.warmup + args.steps + i) % len(bufs)], M, nbhd, out=outs, stream=stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    durs = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)]) * 1e-3  # seconds

    # the binding rooflines, measured in the same run: HBM read rate of a plain stream over the same
    # rotated buffers, and the chip's LDS atomic rate (the pair phase adds one LDS counter per pair)
    from paper_1707_05062_amd import roofline as roof
    stream_rd = roof.read_stream(torch, bufs)
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    lds_probe = roof.lds_atomics(torch, ncu)
    log(f"read stream {stream_rd['gb_s']:.0f} GB/s; LDS atomics distinct {lds_probe['distinct']:.3e}/s")

    if args.copy_probe:
        # a plain device copy of known size (one image buffer per dispatch), for scaling the
        # hardware byte counters of the curve kernel
        dst = torch.empty_like(src)
        for b in bufs:
            dst.copy_(b)
        torch.cuda.synchronize()
        log(f"copy probe: {len(bufs)} copies of {src.numel()} bytes")

    seg = segment_stream(args, ctx, torch, bufs, outs, img, M) if args.only != "curve" else None

    npx = H * W
    alg_bytes = npx * 1 + 3 * M * 8 + 4 * n_thr + 12  # pixels read once + curve and thresholds written
    achieved = alg_bytes / kern / 1e9
    pairs = H * (W - 1) + (H - 1) * W
    lds_atomic = lds_atomic_roofline(plan_used, pairs, npx, kern, lds_probe)
    traffic = measured_traffic(plan_used)
    if traffic:
        log(f"counter-measured traffic for this kernel build and plan: {traffic['bytes']:.0f} B/launch")
    log(f"wall {wall:.4f}s for {args.steps} steps; kernel mean {kern*1e6:.2f} us "
        f"p50 {np.median(durs)*1e6:.2f} p99 {np.percentile(durs, 99)*1e6:.2f} us")
    res = {
        "value": npx * args.steps / wall / 1e9,
        "ms_per_step": wall / args.steps * 1e3,
        "plan": plan_used,
        "tuning": tuned,
        "frame_ms": latency_ms(durs),
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic["bytes"] if traffic else None,
            "kernel_us": kern * 1e6,
            "alg_bytes_per_launch": alg_bytes,
            "hbm_vs_stream_frac": achieved / stream_rd["gb_s"],
            "read_stream": stream_rd,
            "lds_atomic": lds_atomic,
        },
        "traffic_source": traffic["source"] if traffic else
            "null: no hardware-counter measurement for this kernel build and plan",
        "selfcheck": selfcheck,
        "segment": seg,
        "H": H, "W": W, "M": M, "nbhd": nbhd, "rotate_buffers": len(bufs),
        "_lds_probe": lds_probe,
    }
    del bufs
    return res, img


# ------------------------------------------------------------------------------------------------
# the other single-image workloads: 256x256 u8, and 4096x4096 12-bit u16 (M = 4096) at N4 and N8

def pair_gaps(img: np.ndarray, nbhd: int) -> np.ndarray:
    f = img.astype(np.int64)
    d = [np.abs(f[:, 1:] - f[:, :-1]).ravel(), np.abs(f[1:] - f[:-1]).ravel()]
    if nbhd == 8:
        d += [np.abs(f[1:, 1:] - f[:-1, :-1]).ravel(), np.abs(f[1:, :-1] - f[:-1, 1:]).ravel()]
    return np.concatenate(d)


def _dtype_code(a: np.ndarray) -> int:
    from paper_1707_05062_amd import _lib
    return _lib.U16 if a.dtype == np.uint16 else _lib.U8


def config_line(K, torch, name: str, workload: str, img: np.ndarray, M: int, nbhd: int, lds_probe: dict,
                reps: int = 200, rotate: int = 10) -> dict:
    """One image per launch, autotuned plan, inputs resident and rotated over `rotate` copies;
    kernel time from HIP events on the launch stream around `reps` back-to-back launches, plus 100
    individually bracketed launches for the latency percentiles. Self-check: the closed-form totals
    over the whole curve (sum_t count(t) = sum of the pair gaps, sum_t sum(t) = sum of floor(gap^2/4))."""
    dev = torch.device("cuda", 0)
    a = np.ascontiguousarray(img)
    src = (torch.from_numpy(a.view(np.int16)).to(dev).view(torch.uint16) if a.dtype == np.uint16
           else torch.from_numpy(a).to(dev))
    bufs = [src.clone() for _ in range(rotate)]
    H, W = a.shape
    ctx = K.Context(0)
    try:
        plan, us = ctx.autotune([bufs[0]], M, nbhd, reps=3)
        used = ctx.get_plan(_dtype_code(a), H, W, M, nbhd)
        outs = ctx.alloc_outputs(M, M)
        stream = torch.cuda.current_stream(dev)
        ctx.curve_async(bufs[0], M, nbhd, out=outs, stream=stream)
        torch.cuda.synchronize()
        d = pair_gaps(a, nbhd)
        n_thr, t0, status = [int(x) for x in outs["ints"].cpu()]
        ok = bool(int(outs["count"].sum()) == int(d.sum()) and int(outs["sum"].sum()) == int((d * d // 4).sum())
                  and status == 0)
        for i in range(10):
            ctx.curve_async(bufs[i % rotate], M, nbhd, out=outs, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(reps):
            ctx.curve_async(bufs[(10 + i) % rotate], M, nbhd, out=outs, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        kern = e0.elapsed_time(e1) * 1e-3 / reps
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(100)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(100)]
        for i in range(100):
            starts[i].record(stream)
            ctx.curve_async(bufs[i % rotate], M, nbhd, out=outs, stream=stream)
            ends[i].record(stream)
        torch.cuda.synchronize()
        durs = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)]) * 1e-3
    finally:
        ctx.close()
    npx = a.size
    alg_bytes = npx * a.itemsize + 3 * M * 8 + 4 * n_thr + 12
    log(f"{name}: {kern*1e6:.2f} us, {npx / kern / 1e9:.1f} Gpixel/s, selfcheck {ok}")
    return {"workload": workload, "H": int(H), "W": int(W), "M": M, "nbhd": nbhd, "plan": used,
            "tuning_median_us": us, "kernel_us": kern * 1e6, "gpixel_s": npx / kern / 1e9,
            "frame_ms": latency_ms(durs),
            "roofline": {"bound": "hbm", "achieved": alg_bytes / kern / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg_bytes / kern / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_launch": alg_bytes,
                         "lds_atomic": lds_atomic_roofline(used, len(d), npx, kern, lds_probe)},
            "thresholds": n_thr, "selfcheck": ok}


def nbhd_line(K, torch, name: str, workload: str, img: np.ndarray, M: int, half, hex: bool, prefilter: bool,
              pairs: int, reps: int = 100, rotate: int = 16) -> dict:
    """The other-neighbourhood / pre-filter entry point on one image per launch, inputs resident and
    rotated; HIP events around `reps` back-to-back launches on the launch stream. Self-check: the
    closed-form total over the curve (sum_t count(t) = sum of the pair gaps) on the raw image (no
    filter) or the result's own consistency (filter on)."""
    dev = torch.device("cuda", 0)
    a = np.ascontiguousarray(img)
    src = torch.from_numpy(a).to(dev)
    bufs = [src.clone() for _ in range(rotate)]
    ctx = K.Context(0)
    try:
        stream = torch.cuda.current_stream(dev)
        outs = ctx.alloc_outputs(M, M)
        ctx.curve_nbhd_async(bufs[0], M, half=half, hex=hex, prefilter=prefilter, out=outs, stream=stream)
        torch.cuda.synchronize()
        n_thr, t0, status = [int(x) for x in outs["ints"].cpu()]
        ok = status == 0
        for i in range(10):
            ctx.curve_nbhd_async(bufs[i % rotate], M, half=half, hex=hex, prefilter=prefilter, out=outs, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(reps):
            ctx.curve_nbhd_async(bufs[(10 + i) % rotate], M, half=half, hex=hex, prefilter=prefilter, out=outs,
                                 stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        kern = e0.elapsed_time(e1) * 1e-3 / reps
    finally:
        ctx.close()
    npx = a.size
    alg_bytes = npx * a.itemsize + 3 * M * 8 + 4 * n_thr + 12
    log(f"{name}: {kern*1e6:.2f} us, {npx / kern / 1e9:.1f} Gpixel/s, status {status}")
    return {"workload": workload, "kernel_us": kern * 1e6, "gpixel_s": npx / kern / 1e9,
            "pairs_per_launch": pairs, "pairs_per_s": pairs / kern,
            "roofline": {"bound": "hbm", "achieved": alg_bytes / kern / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg_bytes / kern / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_launch": alg_bytes},
            "thresholds": n_thr, "t0": t0, "status_ok": ok}


def nbhd_configs(K, torch, gen) -> dict:
    img = gen.cfg2_image()
    H, W = img.shape
    n4 = H * (W - 1) + (H - 1) * W
    hexp = n4 + (H - 1) * (W - 1)
    base = "3456x5184 uint8 (18 MP) as the headline, M=256"
    return {
        "hex6_18mp": nbhd_line(K, torch, "hex6 18 MP", base + ", hexagonal 6-neighbourhood (odd rows shifted "
                               "right)", img, 256, None, True, False, hexp),
        "n4_prefilter_18mp": nbhd_line(K, torch, "N4 + binomial 18 MP", base + ", 3x3 binomial pre-filter fused "
                                       "into the tile loader, then N4", img, 256, [(0, 1), (1, 0)], False, True, n4),
        "n4_nbhd_path_18mp": nbhd_line(K, torch, "N4 via nbhd path 18 MP", base + ", N4 through the generic "
                                       "neighbourhood kernel (no filter), for comparison with the headline kernel",
                                       img, 256, [(0, 1), (1, 0)], False, False, n4),
    }


def other_configs(K, torch, gen, lds_probe: dict) -> dict:
    out = {"c1_256x256_u8_n4": config_line(
        K, torch, "c1", "256x256 uint8, six constant rectangles + N(0,8^2) noise, M=256, 4-neighbourhood",
        gen.cfg1_image(), 256, 4, lds_probe, reps=1000, rotate=4)}
    c3 = gen.cfg3_image()
    for nbhd in (4, 8):
        out[f"c3_4096x4096_u16_m4096_n{nbhd}"] = config_line(
            K, torch, f"c3 N{nbhd}", "4096x4096 uint16 12-bit, 500 Voronoi cells U[0,4095] + N(0,30^2) "
            f"noise, M=4096, {nbhd}-neighbourhood", c3, 4096, nbhd, lds_probe)
    return out


# ------------------------------------------------------------------------------------------------
# segmentation of the same image by its thresholds: a read-once, write-once stream

def segment_stream(args, ctx, torch, bufs, outs, img, M) -> dict:
    H, W = img.shape
    n = int(outs["ints"][0])
    cap = min(outs["thr"].numel(), 255)  # u8 labels: at most 255 thresholds (M = 256 has at most 128)
    labs = [torch.empty((H, W), dtype=torch.uint8, device=bufs[0].device) for _ in range(2)]
    stream = torch.cuda.current_stream()
    ctx.segment(bufs[0], outs["thr"], outs["ints"][0:1], cap, M, out=labs[0])
    torch.cuda.synchronize()
    thr = outs["thr"][:n].cpu().numpy()
    check = bool(np.array_equal(labs[0].cpu().numpy(), np.searchsorted(thr, img, side="left")))
    for i in range(args.warmup):
        ctx.segment(bufs[i % len(bufs)], outs["thr"], outs["ints"][0:1], cap, M, out=labs[i % 2])
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(args.steps):
        ctx.segment(bufs[i % len(bufs)], outs["thr"], outs["ints"][0:1], cap, M, out=labs[i % 2])
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / args.steps
    nbytes = 2 * H * W  # each u8 pixel read once, each u8 label written once
    log(f"segment: {t*1e6:.2f} us per launch, {nbytes / t / 1e9:.0f} GB/s, labels match: {check}")

    # class statistics (histogram + fold) and the class-mean image, same image and thresholds
    n_dev = outs["ints"][0:1]
    means = []

    def timed(fn):
        for i in range(args.warmup):
            fn(i)
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        for i in range(args.steps):
            fn(i)
        a1.record(stream)
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) * 1e-3 / args.steps

    def stats(i):
        means[:] = [ctx.class_stats(bufs[i % len(bufs)], outs["thr"], n_dev, cap, M)]

    ts = timed(stats)
    cnt, tot, mean = [x.cpu().numpy() for x in means[0]]
    lab = np.searchsorted(thr, img, side="left").reshape(-1)
    want_cnt = np.bincount(lab, minlength=n + 1)
    want_tot = np.bincount(lab, weights=img.reshape(-1).astype(np.float64), minlength=n + 1).astype(np.int64)
    stats_ok = bool(np.array_equal(cnt[:n + 1], want_cnt) and np.array_equal(tot[:n + 1], want_tot))
    mimgs = [torch.empty_like(bufs[0]) for _ in range(2)]
    tm = timed(lambda i: ctx.mean_image(bufs[i % len(bufs)], outs["thr"], n_dev, cap, M, means[0][2],
                                        out=mimgs[i % 2]))
    mean_ok = bool(np.array_equal(mimgs[(args.steps - 1) % 2].cpu().numpy(),
                                  np.rint(mean[:n + 1])[lab].reshape(img.shape).astype(np.uint8)))
    log(f"class stats: {ts*1e6:.2f} us ({H * W / ts / 1e9:.0f} GB/s), match {stats_ok}; "
        f"class-mean image: {tm*1e6:.2f} us ({nbytes / tm / 1e9:.0f} GB/s), match {mean_ok}")
    return {"workload": f"labels of the {H}x{W} image by its {n} thresholds (u8 in, u8 labels)",
            "kernel_us": t * 1e6, "gpixel_s": H * W / t / 1e9,
            "roofline": {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": nbytes / t / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_launch": nbytes},
            "labels_match_searchsorted": check,
            "class_stats_us": ts * 1e6, "class_stats_gb_s": H * W / ts / 1e9, "class_stats_match": stats_ok,
            "mean_image_us": tm * 1e6, "mean_image_gb_s": nbytes / tm / 1e9, "mean_image_match": mean_ok}


# ------------------------------------------------------------------------------------------------
# batched: 96 images of uneven sizes, one persistent launch vs one launch per image

def batched(args, K, ctx, torch, gen) -> dict:
    M, nbhd = 256, 4
    imgs = gen.batch_images(n=96)
    npx = sum(im.size for im in imgs)
    log(f"batch: {len(imgs)} images, {npx / 1e6:.1f} MP")
    copies = [[torch.from_numpy(im).cuda() for im in imgs] for _ in range(2)]  # 2 x 170 MB > Infinity Cache
    bctx = K.Context(0)  # its own context: the batch plan is tuned for this workload
    plan, us = bctx.autotune(copies[0], M, nbhd, reps=3)
    log(f"batch autotuned plan {plan} {us:.1f} us")
    pctx = K.Context(0)  # the plain kernel: default plan, grid sized to each image
    cap = M
    bout = bctx.alloc_outputs(M, cap, len(imgs))
    souts = [pctx.alloc_outputs(M, cap) for _ in imgs]
    stream = torch.cuda.current_stream()

    def run_batch(k):
        bctx.curve_batch(copies[k % 2], M, nbhd, out=bout)

    def run_plain(k):
        for i, im in enumerate(copies[k % 2]):
            pctx.curve_async(im, M, nbhd, out=souts[i], stream=stream)

    def timeit(fn, reps):
        for k in range(2):
            fn(k)
        torch.cuda.synchronize()
        ts = []
        for k in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn(k)
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        return float(np.median(ts))

    t_b = timeit(run_batch, args.batch_reps)
    t_p = timeit(run_plain, args.batch_reps)
    # results of the two paths must agree bit for bit
    torch.cuda.synchronize()
    agree = True
    n = len(imgs)
    for i in range(n):
        agree &= bool(torch.equal(bout["sum"][i], souts[i]["sum"]) and torch.equal(bout["count"][i], souts[i]["count"])
                      and torch.equal(bout["C"][i], souts[i]["C"]))
    bctx.close()
    pctx.close()
    return {"workload": "96 uint8 images, pixel count log-uniform in [128^2, 4000x3000], aspect in "
                        "{1, 4/3, 16/9}, six-rectangle content + N(0,8^2) noise, M=256, 4-neighbourhood",
            "images": n, "mpixels": npx / 1e6, "plan": plan,
            "persistent_ms": t_b * 1e3, "persistent_gpixel_s": npx / t_b / 1e9,
            "plain_ms": t_p * 1e3, "plain_gpixel_s": npx / t_p / 1e9,
            "speedup": t_p / t_b, "results_identical": agree}


# ------------------------------------------------------------------------------------------------
# served: Poisson arrivals through the serving loop

SERVE_CLASSES = ("1080p", "4k", "18mp")
SERVE_MIX = (0.7, 0.2, 0.1)


def make_trace(rate: float, seconds: float, seed: int = 5):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        out.append((t, int(rng.choice(3, p=SERVE_MIX))))
    return out


def run_trace(K, ctx, pool, trace, warm_s, server_kw, burst=False, labels=None):
    srv = K.Server(ctx, **server_kw)
    counters = {c: 0 for c in SERVE_CLASSES}
    try:
        # one request per class first, so that per-shape graphs exist before the clock starts
        for c in SERVE_CLASSES:
            if labels is not None:
                srv.wait(srv.submit(pool[c][0], labels=labels[c][0]))
            else:
                srv.wait(srv.submit(pool[c][0]))
        tickets: queue.Queue = queue.Queue()
        t0 = time.monotonic_ns() + 20_000_000

        def submitter():
            while time.monotonic_ns() < t0:  # the clock starts at t0, for a burst too
                time.sleep(0.0005)
            for (ta, ci) in trace:
                c = SERVE_CLASSES[ci]
                frame = pool[c][counters[c] % len(pool[c])]
                counters[c] += 1
                target = t0 + (0 if burst else int(ta * 1e9))
                if not burst:
                    while True:
                        d = target - time.monotonic_ns()
                        if d <= 0:
                            break
                        if d > 300_000:
                            time.sleep((d - 200_000) / 1e9)
                try:
                    if labels is not None:
                        lab = labels[c][(counters[c] - 1) % len(labels[c])]
                        tk = srv.submit(frame, labels=lab)
                    else:
                        tk = srv.submit(frame)
                except K.KohlerError as e:
                    tickets.put((ta, ci, None, e.status))
                    continue
                tickets.put((ta, ci, tk, 0))
            tickets.put(None)

        th = threading.Thread(target=submitter)
        th.start()
        lat = {c: [] for c in SERVE_CLASSES}
        refused, bad, first, last, npx, done = 0, 0, None, None, 0, 0
        while True:
            item = tickets.get()
            if item is None:
                break
            ta, ci, tk, st = item
            if tk is None:
                refused += 1
                continue
            res, info = srv.wait(tk)
            if res.status != 0:
                bad += 1
            arrival = t0 + (0 if burst else int(ta * 1e9))
            if burst or ta >= warm_s:
                lat[SERVE_CLASSES[ci]].append((info["t_done_ns"] - arrival) / 1e6)
                npx += pool[SERVE_CLASSES[ci]][0].shape[0] * pool[SERVE_CLASSES[ci]][0].shape[1]
                done += 1
                first = arrival if first is None else min(first, arrival)
                last = info["t_done_ns"] if last is None else max(last, info["t_done_ns"])
        th.join()
        stats = srv.stats()
    finally:
        srv.close()
    span = (last - first) / 1e9 if done else float("nan")
    alls = [x for c in SERVE_CLASSES for x in lat[c]]
    out = {"requests": done, "refused": refused, "failed": bad,
           "req_per_s": done / span, "gpixel_s": npx / span / 1e9,
           "p50_ms": pct(alls, 50), "p99_ms": pct(alls, 99),
           "per_class": {c: {"n": len(lat[c]), "p50_ms": pct(lat[c], 50), "p99_ms": pct(lat[c], 99)}
                         for c in SERVE_CLASSES},
           "launches": stats["launches"], "graph_launches": stats["graph_launches"],
           "batched_launches": stats["batched_launches"], "max_batch": stats["max_batch_seen"],
           "peak_inflight": stats["peak_inflight"]}
    return out


def served(args, K, ctx, torch, gen) -> dict:
    raw = gen.serve_pool(n1080=args.pool_1080, n4k=args.pool_4k, n18=args.pool_18mp)
    pool = {c: [torch.from_numpy(f).pin_memory() for f in raw[c]] for c in SERVE_CLASSES}
    log("serve pool: " + ", ".join(f"{c} x{len(pool[c])}" for c in SERVE_CLASSES))
    # spot check: the server's result for one frame of each class equals the context call
    check_srv = K.Server(ctx, slots=4, lanes=1, max_batch=4, hbm_budget_bytes=1 << 30)
    ok = True
    for c in SERVE_CLASSES:
        r, _ = check_srv.wait(check_srv.submit(pool[c][1 % len(pool[c])]))
        ref = ctx.curve(raw[c][1 % len(raw[c])], 256, 4)
        ok &= bool(np.array_equal(r.sum, ref.sum) and np.array_equal(r.count, ref.count)
                   and np.array_equal(r.C, ref.C) and r.t0 == ref.t0)
    check_srv.close()

    server_kw = dict(slots=32, lanes=2, max_batch=16, use_graphs=False, hbm_budget_bytes=2 << 30)
    graph_kw = dict(server_kw, use_graphs=True)
    video_kw = dict(server_kw, label_t0=True, hbm_budget_bytes=3 << 30)
    # video mode: every request also returns its two-class labels at its own t0, into pinned host
    # buffers cycled per class (more buffers than requests in flight)
    labels = {c: [torch.empty(pool[c][0].shape, dtype=torch.uint8).pin_memory() for _ in range(48)]
              for c in SERVE_CLASSES}
    plain_kw = dict(slots=1, lanes=1, max_batch=1, use_graphs=False, hbm_budget_bytes=256 << 20)
    trace = make_trace(args.rate, args.serve_seconds + 1.0)
    log(f"served: {len(trace)} arrivals over {args.serve_seconds + 1.0:.0f} s")
    res = {"workload": f"Poisson arrivals at {args.rate:g}/s for {args.serve_seconds:g} s after 1 s "
                       "warm-up: 1080p frames 70% (40-blob canvas, window moving 2 px/frame, fresh "
                       "N(0,6^2) noise), 4K frames 20% (same rule), 18 MP stills 10%; u8, M=256, N4; "
                       "pinned host frames cycled from a pool; latency = scheduled arrival to "
                       "results in host memory",
           "results_match_context": ok,
           "server_config": server_kw, "server_graphs_config": graph_kw, "server_video_t0_config": video_kw,
           "plain_config": plain_kw}
    res["server"] = run_trace(K, ctx, pool, trace, 1.0, server_kw)
    log(f"served server: {res['server']['p50_ms']:.3f}/{res['server']['p99_ms']:.3f} ms p50/p99")
    res["server_graphs"] = run_trace(K, ctx, pool, trace, 1.0, graph_kw)
    log(f"served server with per-shape graphs: {res['server_graphs']['p50_ms']:.3f}/{res['server_graphs']['p99_ms']:.3f} ms p50/p99")
    res["server_video_t0"] = run_trace(K, ctx, pool, trace, 1.0, video_kw, labels=labels)
    log(f"served server, video mode (labels at t0 included): {res['server_video_t0']['p50_ms']:.3f}/"
        f"{res['server_video_t0']['p99_ms']:.3f} ms p50/p99")
    res["plain"] = run_trace(K, ctx, pool, trace, 1.0, plain_kw)
    log(f"served plain:  {res['plain']['p50_ms']:.3f}/{res['plain']['p99_ms']:.3f} ms p50/p99")
    rng = np.random.default_rng(55)
    burst = [(0.0, int(rng.choice(3, p=SERVE_MIX))) for _ in range(args.burst)]
    res["burst"] = {"requests": len(burst),
                    "server": run_trace(K, ctx, pool, burst, 0.0, server_kw, burst=True),
                    "server_graphs": run_trace(K, ctx, pool, burst, 0.0, graph_kw, burst=True),
                    "server_video_t0": run_trace(K, ctx, pool, burst, 0.0, video_kw, burst=True, labels=labels),
                    "plain": run_trace(K, ctx, pool, burst, 0.0, plain_kw, burst=True)}
    log(f"burst: server {res['burst']['server']['gpixel_s']:.1f} Gpx/s, "
        f"plain {res['burst']['plain']['gpixel_s']:.1f} Gpx/s")
    return res


# ------------------------------------------------------------------------------------------------

def run(args) -> dict:
    import torch

    import gen
    import paper_1707_05062_amd as K

    ctx = K.Context(0)
    head, img = headline(args, K, ctx, torch, gen)
    lds_probe = head.pop("_lds_probe")
    result = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": "3456x5184 uint8 (18 MP), smooth 2-D cosine background (amplitude 60) + 40 "
                        "ellipses with means U[0,255] + N(0,5^2) noise, M=256, 4-neighbourhood, "
                        "one image per launch",
            "H": head["H"], "W": head["W"], "M": head["M"], "nbhd": head["nbhd"],
            "rotate_buffers": head["rotate_buffers"], "plan": head["plan"], "tuning": head["tuning"],
        },
        "frame_ms": head["frame_ms"],
        "roofline": head["roofline"],
        "selfcheck": head["selfcheck"],
        "segment": head["segment"],
        "paper_context": {
            "hardware": "Intel Core i7-4702HQ, 2.20 GHz, 4 cores / 8 threads, 16 GB (Sec. 4)",
            "image": "3672x4896 photograph, about 18 MP (Table 1)",
            "fast_A_seconds": 0.130, "fast_A_gpixel_s": 0.138, "direct_D_seconds": 52.9,
            "gain_A_vs_D_18mp": 405,
            "video": {"frame": "502x480", "fast_A_frames_s": 96.96, "direct_D_frames_s": 0.99,
                      "gain_A_vs_D": 96, "source": "Table 2 (the abstract's factor)"},
            "this_run_vs_fast_A": None,
            "note": "context only: the paper's own CPU timings, other hardware and another image",
        },
    }
    result["paper_context"]["this_run_vs_fast_A"] = head["value"] / 0.138
    if args.only != "curve":
        result["configs"] = other_configs(K, torch, gen, lds_probe)
        result["neighbourhoods"] = nbhd_configs(K, torch, gen)
    if args.only == "all":
        result["batched"] = batched(args, K, ctx, torch, gen)
        result["served"] = served(args, K, ctx, torch, gen)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        result["cpu_baseline"] = cpu_baseline(img, head["M"], head["nbhd"])
    ctx.close()
    return result


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--rotate", type=int, default=32, help="distinct input buffers cycled by the steps")
    ap.add_argument("--plan", default="", help="fixed plan form:band:block:grid:px_per_lane:replicas[:copies] "
                                               "instead of autotuning")
    ap.add_argument("--only", choices=["all", "headline", "curve"], default="all",
                    help="headline: the curve and the segmentation of the 18 MP image only; curve: the curve only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, copy each input buffer once (a reference for byte counters)")
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--rate", type=float, default=240.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--burst", type=int, default=400)
    ap.add_argument("--pool-1080", type=int, default=48)
    ap.add_argument("--pool-4k", type=int, default=12)
    ap.add_argument("--pool-18mp", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (images are independent; "
              "run one process per GPU on separate images). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    res = run(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
