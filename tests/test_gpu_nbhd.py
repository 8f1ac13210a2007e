"""GPU parity for other neighbourhoods and the pre-filter (kohler_curve_nbhd_async) against the CPU
oracle: a symmetric structuring element given by its half, the hexagonal 6-neighbourhood (odd rows
shifted right by half a pixel), each with and without the 3x3 binomial low-pass applied first.

Sizes run from every shape up to 6x6 through multi-tile images with ragged edges (tiles are 512
columns by up to 16 rows) to the 18 MP workload; sum and count bit-exact, C to 0 ulp, thresholds and
t0 identical."""
import numpy as np
import pytest

import _pins
import gen
import oracle
from _gpu import assert_same, say, to_device

pytestmark = pytest.mark.gpu

N4_HALF = [(0, 1), (1, 0)]
N8_HALF = N4_HALF + [(1, 1), (1, -1)]


@pytest.fixture(scope="module")
def K():
    import paper_1707_05062_amd as K
    return K


@pytest.fixture(scope="module")
def ctx(K):
    c = K.Context(0)
    yield c
    c.close()


def reference_nbhd(img, M, half=None, hex=False, prefilter=False, exact_all=True):
    f = oracle.binomial3(img) if prefilter else np.asarray(img)
    if exact_all:
        s, k, _ = oracle.curve_nbhd(f, M, offsets=None if hex else oracle.full_of(half), hex=hex)
    else:
        s, k = oracle.alg1_nbhd(f, M, half=None if hex else half, hex=hex)
    c = np.where(k > 0, s.astype(np.float64) / np.where(k > 0, k, 1).astype(np.float64), 0.0)
    thr, t0, _, n = oracle.thresholds(s, k)
    return dict(sum=s, count=k, C=c, thr=thr, t0=t0, n=n)


def check(ctx, img, M, half=None, hex=False, prefilter=False, what="", exact_all=True):
    res = ctx.curve_nbhd(to_device(img), M, half=half, hex=hex, prefilter=prefilter)
    ref = reference_nbhd(img, M, half, hex, prefilter, exact_all)
    assert_same(res.sum, res.count, res.C, res.thresholds, res.t0, res.n_thresholds, ref, what=what)
    return res


def test_hand_fixtures(ctx):
    for name in _pins.nbhd_fixture_names():
        fx = _pins.load_nbhd_fixture(name)
        half = None if fx["hex"] else oracle.half_of(fx["offsets"])
        res = ctx.curve_nbhd(to_device(fx["image"].astype(np.uint8)), fx["M"], half=half, hex=fx["hex"])
        assert list(res.sum) == list(fx["sum"]) and list(res.count) == list(fx["count"]), name
        assert list(res.thresholds) == fx["thresholds"] and res.t0 == fx["t0"], name


def test_tiny_exhaustive(ctx):
    rng = np.random.default_rng(61)
    halves = [None, N4_HALF, N8_HALF, [(0, 2), (1, -3)], [(2, 1)]]
    n = 0
    for H in range(1, 7):
        for W in range(1, 7):
            for M in (2, 5, 256):
                img = rng.integers(0, M, size=(H, W)).astype(np.uint8)
                for half in halves:
                    for pf in (False, True):
                        check(ctx, img, M, half=half, hex=half is None, prefilter=pf,
                              what=f"{H}x{W} M={M} {half or 'hex'} pf={pf}")
                        n += 1
    say("tiny cases", n)


def test_reduces_to_main_kernel(ctx):
    """The offset sets of N4 and N8 through this path give the main kernel's curves."""
    rng = np.random.default_rng(62)
    for shape in [(37, 301), (129, 1100), (17, 513)]:
        img = gen.random_image(rng, *shape, 256, np.uint8, "smooth")
        dev = to_device(img)
        for half, nbhd in ((N4_HALF, 4), (N8_HALF, 8)):
            a = ctx.curve_nbhd(dev, 256, half=half)
            b = ctx.curve(dev, 256, nbhd)
            assert np.array_equal(a.sum, b.sum) and np.array_equal(a.count, b.count)
            assert np.array_equal(a.C, b.C) and list(a.thresholds) == list(b.thresholds) and a.t0 == b.t0


# (60, 1600): interior tiles (every neighbour of every pixel inside the image, pairs taken without
# tests) next to border tiles on all four sides, for every radius up to 7
@pytest.mark.parametrize("shape", [(1, 1000), (1000, 1), (37, 301), (64, 512), (17, 1025), (129, 513), (60, 1600)])
def test_ragged_u8(ctx, shape):
    rng = np.random.default_rng(sum(shape))
    for kind in ("uniform", "smooth"):
        img = gen.random_image(rng, *shape, 256, np.uint8, kind)
        half = _pins.random_half(rng, n_max=6, r=7)
        for hx, hf in ((True, None), (False, half)):
            for pf in (False, True):
                check(ctx, img, 256, half=hf, hex=hx, prefilter=pf, what=f"{shape} {kind} {hf or 'hex'} pf={pf}")
        # a small M with clamping (M < 256 on 8-bit pixels)
        small = np.minimum(img, 36)
        check(ctx, small, 37, hex=True, what=f"{shape} M=37 hex")


@pytest.mark.parametrize("shape", [(37, 301), (64, 1100)])
def test_ragged_u16(ctx, shape):
    rng = np.random.default_rng(7 * sum(shape))
    for M in (700, 4096, 8192):
        img = gen.random_image(rng, *shape, M, np.uint16, "smooth")
        half = _pins.random_half(rng, n_max=5, r=4)
        for hx, hf in ((True, None), (False, half)):
            for pf in (False, True):
                check(ctx, img, M, half=hf, hex=hx, prefilter=pf, what=f"u16 {shape} M={M} {hf or 'hex'} pf={pf}")


def test_cfg2_full_size(ctx):
    """18 MP: the hexagonal grid, and N4 after the pre-filter, against Algorithm 1 over the half;
    eight thresholds against the brute force itself."""
    img = gen.cfg2_image()
    ts = np.array([0, 20, 54, 100, 128, 200, 254, 255], np.int32)
    for hx, half, pf in ((True, None, False), (False, N4_HALF, True)):
        res = check(ctx, img, 256, half=half, hex=hx, prefilter=pf, exact_all=False, what=f"cfg2 {half or 'hex'} pf={pf}")
        f = oracle.binomial3(img) if pf else img
        s, k, c = oracle.curve_nbhd(f, 256, offsets=None if hx else oracle.full_of(half), hex=hx, ts=ts)
        assert np.array_equal(res.sum[ts], s) and np.array_equal(res.count[ts], k) and np.array_equal(res.C[ts], c)
        say("cfg2", "hex" if hx else "N4 prefiltered", res.n_thresholds, res.t0)


def test_range_error(ctx, K):
    img = gen.cfg1_image()
    bad = img.copy()
    bad[7, 9] = 200
    for pf in (False, True):
        res = ctx.curve_nbhd(to_device(bad), 150, hex=True, prefilter=pf, check=False)
        assert res.status == K.E_RANGE
    ok = np.minimum(img, 149)
    check(ctx, ok, 150, hex=True, what="after range error")


def test_bad_arguments(ctx, K):
    dev = to_device(gen.cfg1_image())
    for half in ([], [(0, 0)], [(0, 1), (0, -1)], [(8, 0)], [(0, 1)] * 17, [(1, 2), (1, 2)]):
        with pytest.raises((K.KohlerError, ValueError)):
            ctx.curve_nbhd(dev, 256, half=half)
    with pytest.raises(K.KohlerError):
        ctx.curve_nbhd(to_device(np.zeros((4, 4), np.uint16)), 8193, hex=True)
