"""Per-phase breakdown of one curve launch, from the measurement build ``libkohler_phase.so``.

Build it first on the CPU (``python -m paper_1707_05062_amd.build --phase-clock``), then run
``python -m paper_1707_05062_amd.phase_clock`` on the GPU. Every workgroup of the curve kernel
records the 100 MHz real-time counter at its phase boundaries (entry, LDS tables cleared, pair work
done, merge atomics issued, merge atomics performed, ticket taken; the finishing workgroup also after
gathering the accumulator replicas and at its end) and each wave the end of its pair work. The script
launches the kernel on the 3456x5184 u8 image (M = 256, N4), or the 4096x4096 12-bit image (M = 4096,
N4 or N8), over rotated buffers, reads the stamps after each launch and prints a Markdown summary
(medians over the launches, in microseconds). For M > 256 the finishing workgroup sums the replicas
level block by level block inside its scan, so its gather time is part of its finish.
"""
from __future__ import annotations

import argparse
import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SLOTS, MAXWG, WAVES = 16, 4096, 16
TICK_US = 0.01  # the real-time counter runs at 100 MHz


def breakdown(slots: np.ndarray, waves: np.ndarray, grid: int, nwaves: int) -> dict:
    s = slots.reshape(MAXWG, SLOTS)[:grid].astype(np.int64)
    w = waves.reshape(MAXWG, WAVES)[:grid, :nwaves].astype(np.int64)
    fin = np.nonzero(s[:, 7])[0]
    assert len(fin) == 1, f"expected one finishing workgroup, found {len(fin)}"
    f = int(fin[0])
    t0 = s[:, 0].min()
    us = lambda x: float(x) * TICK_US  # noqa: E731
    # placement: compute unit = (XCD, engine, shader array, unit) from the hardware id registers
    hw, xcc = s[:, 8], s[:, 9]
    cu = (xcc & 0xF) * 4096 + ((hw >> 13) & 7) * 512 + ((hw >> 12) & 1) * 256 + ((hw >> 8) & 0xF)
    _, per_cu = np.unique(cu, return_counts=True)
    return {
        "compute_units_used": float(len(per_cu)),
        "max_workgroups_per_cu": float(per_cu.max()),
        "span": us(s[f, 7] - t0),
        "dispatch_spread": us(s[:, 0].max() - t0),
        "clear": us(np.median(s[:, 1] - s[:, 0])),
        "pairs_median": us(np.median(s[:, 2] - s[:, 1])),
        "pairs_max": us((s[:, 2] - s[:, 1]).max()),
        "wave_spread_median": us(np.median(w.max(1) - w.min(1))),
        "all_pairs_done": us(s[:, 2].max() - t0),
        "project_median": us(np.median(s[:, 3] - s[:, 2])),
        "atomics_median": us(np.median(s[:, 4] - s[:, 3])),
        "ticket_median": us(np.median(s[:, 5] - s[:, 4])),
        "last_pairs_to_ticket": us(s[f, 5] - s[:, 2].max()),
        "fin_project": us(s[f, 3] - s[f, 2]),
        "fin_atomics": us(s[f, 4] - s[f, 3]),
        "fin_ticket": us(s[f, 5] - s[f, 4]),
        "fin_gather": us(s[f, 6] - s[f, 5]),
        "fin_finish": us(s[f, 7] - s[f, 6]),
        "fin_finish_cycles": float(s[f, 11] - s[f, 10]),
        "fin_cycles_scan": float(s[f, 12] - s[f, 10]),
        "fin_cycles_compare": float(s[f, 13] - s[f, 12]),
        "fin_cycles_maxima": float(s[f, 14] - s[f, 13]),
        "fin_cycles_out": float(s[f, 11] - s[f, 14]),
        "fin_wg_pairs_end_rank": int((s[:, 2] <= s[f, 2]).sum()),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--plan", default="1:31:1024:256:8:8:4", help="form:band:block:grid:px_per_lane:replicas[:copies]")
    ap.add_argument("--launches", type=int, default=30)
    ap.add_argument("--rotate", type=int, default=32)
    ap.add_argument("--lib", default="", help="another measurement build of the library (default: libkohler_phase.so)")
    ap.add_argument("--workload", choices=["18mp", "c3n4", "c3n8", "nbhd18mp"], default="18mp",
                    help="18mp: the 3456x5184 u8 image, M=256, N4; c3n4 / c3n8: the 4096x4096 12-bit image, "
                         "M=4096, N4 / N8; nbhd18mp: the 18 MP image through the neighbourhood kernel (N4 "
                         "given by its half offsets; --plan is ignored)")
    args = ap.parse_args()

    import torch

    import gen
    import paper_1707_05062_amd as K
    from paper_1707_05062_amd import _lib
    from paper_1707_05062_amd.build import PHASE_LIB

    ctx = K.Context(0, lib_path=args.lib or PHASE_LIB)
    lib = ctx._lib
    lib.kohler_phase_clock_read.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    lib.kohler_phase_clock_read.restype = ctypes.c_int
    keys = ("form", "band", "block", "grid", "px_per_lane", "replicas", "copies")
    plan = dict(zip(keys, (int(x) for x in args.plan.split(":"))))
    nbhd_path = args.workload == "nbhd18mp"
    if args.workload in ("18mp", "nbhd18mp"):
        img, dt, M, nb = gen.cfg2_image(), _lib.U8, 256, 4
    else:
        img, dt, M, nb = gen.cfg3_image(), _lib.U16, 4096, int(args.workload[-1])
    H, W = img.shape
    if nbhd_path:
        used = {"kernel": "nbhd_kernel", "half": [(0, 1), (1, 0)], "block": 512}
    else:
        ctx.set_plan(dt, M, nb, **plan)
        used = ctx.get_plan(dt, H, W, M, nb)

    def launch(buf):
        if nbhd_path:
            ctx.curve_nbhd_async(buf, M, half=[(0, 1), (1, 0)], out=out)
        else:
            ctx.curve_async(buf, M, nb, out=out)
    dev = torch.device("cuda", 0)
    src = (torch.from_numpy(img.view(np.int16)).to(dev).view(torch.uint16) if img.dtype == np.uint16
           else torch.from_numpy(img).to(dev))
    bufs = [src.clone() for _ in range(min(args.rotate, 8 if img.dtype == np.uint16 else args.rotate))]
    out = ctx.alloc_outputs(M, M)
    slots = np.zeros(MAXWG * SLOTS, np.uint64)
    waves = np.zeros(MAXWG * WAVES, np.uint64)
    for i in range(10):
        launch(bufs[i % len(bufs)])
    torch.cuda.synchronize()
    rows = []
    for i in range(args.launches):
        assert lib.kohler_phase_clock_read(None, None, 1) == 0
        launch(bufs[(10 + i) % len(bufs)])
        torch.cuda.synchronize()
        assert lib.kohler_phase_clock_read(slots.ctypes.data, waves.ctypes.data, 0) == 0
        # workgroups of the launch: those that stamped their entry
        grid = used["grid"] if not nbhd_path else int(np.count_nonzero(slots.reshape(MAXWG, SLOTS)[:, 0]))
        rows.append(breakdown(slots, waves, grid, used["block"] // 64))
        print(f"launch {i}: span {rows[-1]['span']:.2f} us", file=sys.stderr, flush=True)
    assert int(out["ints"][2]) == 0
    med = {k: float(np.median([r[k] for r in rows])) for k in rows[0]}
    print(f"plan {used}; {args.launches} launches of the {H}x{W} {img.dtype} image (M={M}, N{nb}); "
          "medians over launches, microseconds")
    print("| quantity | us |\n|---|---|")
    for k, v in med.items():
        print(f"| {k} | {v:.2f} |")
    ctx.close()


if __name__ == "__main__":
    main()
