#!/usr/bin/env python3
"""Benchmark of the Köhler contrast curve on one MI355X.

Default workload (one "step" = the whole hot path for one image: pair formation, per-pair
accumulation, merge, prefix sums, FP64 division, local maxima and t0, all in one launch):
  cfg2 - a 3456x5184 (about 18 MP) uint8 synthetic image, M = 256, 4-neighbourhood.
The image is resident in HBM before the timed region; the timed steps rotate over --rotate
distinct copies (32 x 17.9 MB = 573 MB) so that the 256 MB Infinity Cache cannot serve them.

Prints ONE JSON line (rank 0) with the throughput in Gpixel/s, the roofline of the kernel
(algorithmic bytes / average kernel duration from HIP events on the launch stream) and the CPU
oracle's throughput on the host cores (the CPU baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E datasheet peak
METRIC = "Gpixel/s for Köhler C(t) curve (18MP, M=256) + % HBM roofline; p50/p99 frame ms"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(img: np.ndarray, M: int, nbhd: int) -> dict:
    """The oracle (plain brute force of eqs (1)-(3), OpenMP over thresholds) on the host cores."""
    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t = time.perf_counter()
    oracle.curve(img, M, nbhd)
    dt = time.perf_counter() - t
    return {"value": img.size / dt / 1e9, "unit": "Gpixel/s", "cores": cores, "kind": "oracle",
            "seconds": dt,
            "sample": f"the full {img.shape[0]}x{img.shape[1]} image, all {M} thresholds, one run"}


def run(args) -> dict:
    import torch

    import gen
    import paper_1707_05062_amd as K

    cfg = gen.CONFIGS["cfg2"]
    H, W, M, nbhd = cfg["H"], cfg["W"], cfg["M"], 4
    img = gen.cfg2_image()
    log(f"cfg2 generated {img.shape}")
    dev = torch.device("cuda", 0)
    src = torch.from_numpy(img).to(dev)
    bufs = [src.clone() for _ in range(max(1, args.rotate))]
    ctx = K.Context(0)
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
    log(f"selfcheck={selfcheck} thresholds={n_thr} t0={t0} plan={ctx.get_plan(1, H, W, M, nbhd)}")

    for i in range(args.warmup):
        ctx.curve_async(bufs[i % len(bufs)], M, nbhd, out=outs)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        ctx.curve_async(bufs[i % len(bufs)], M, nbhd, out=outs)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_begin
    durs = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)]) * 1e-3  # seconds

    npx = H * W
    ms_per_step = wall / args.steps * 1e3
    value = npx * args.steps / wall / 1e9
    kern = float(durs.mean())
    alg_bytes = npx * 1 + 3 * M * 8 + 4 * n_thr + 12  # pixels read once + curve and thresholds written
    achieved = alg_bytes / kern / 1e9
    log(f"wall {wall:.4f}s for {args.steps} steps; kernel mean {kern*1e6:.2f} us "
        f"p50 {np.median(durs)*1e6:.2f} p99 {np.percentile(durs, 99)*1e6:.2f} us")

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": "cfg2: 3456x5184 uint8, smooth cosine background + 40 ellipses + N(0,5^2) noise, "
                        "M=256, 4-neighbourhood, one image per launch",
            "H": H, "W": W, "M": M, "nbhd": nbhd, "rotate_buffers": len(bufs),
            "plan": ctx.get_plan(1, H, W, M, nbhd),
        },
        "frame_ms": {"p50": float(np.median(durs) * 1e3), "p99": float(np.percentile(durs, 99) * 1e3)},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel_us": kern * 1e6,
            "alg_bytes_per_launch": alg_bytes,
        },
        "selfcheck": selfcheck,
        "paper_context": {"fast_A_gpixel_s": 0.138, "hardware": "Intel i7-4702HQ 4C/8T",
                          "image": "3672x4896 photograph (Table 1)"},
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        result["cpu_baseline"] = cpu_baseline(img, M, nbhd)
    ctx.close()
    return result


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--rotate", type=int, default=32, help="distinct input buffers cycled by the steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (images are independent; "
              "run one process per GPU on separate images). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    res = run(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
