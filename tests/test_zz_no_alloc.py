"""The entry point that allocates nothing (kohler_curve_noalloc) against kohler_curve_async.

Both run the same kernels on the same image; the no-allocation call keeps its scratch in the
library's per-GPU device array. Two calls in a row, the second on a smaller image, must each equal
the context's call bit for bit (sum, count, C, thresholds, their number, t0, status)."""
from __future__ import annotations

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def _host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b, what):
    for k in ("sum", "count", "C", "ints"):
        assert np.array_equal(a[k], b[k]), f"{what}: {k} differs"
    n = int(a["ints"][0])
    cap = a["thr"].shape[0]
    assert np.array_equal(a["thr"][:min(n, cap)], b["thr"][:min(n, cap)]), f"{what}: thresholds differ"


@pytest.mark.parametrize("dtype,M,nbhd", [("u8", 256, 4), ("u8", 256, 8), ("u16", 4096, 4)])
def test_noalloc_two_calls_match_async(dtype, M, nbhd):
    import torch

    import paper_1707_05062_amd as K
    ctx = K.Context(0)
    if dtype == "u8":
        big = gen.cfg1_image()
    else:
        rng = np.random.default_rng(11)
        big = rng.integers(0, M, size=(300, 257)).astype(np.uint16)
    small = np.ascontiguousarray(big[37:137, 11:88])  # 100 x 77, a ragged strip
    for img, what in ((big, "first call"), (small, "second call, smaller image")):
        dev = torch.from_numpy(img).to("cuda:0")
        cap = M // 2 + 1  # room for every local maximum
        a = ctx.curve_async(dev, M, nbhd, capacity=cap)
        b = K.curve_noalloc(dev, M, nbhd, capacity=cap)
        torch.cuda.synchronize()
        ha, hb = _host(a), _host(b)
        assert int(ha["ints"][2]) == 0 and int(hb["ints"][2]) == 0
        _same(ha, hb, f"{dtype} M={M} N{nbhd} {what}")
    ctx.close()
