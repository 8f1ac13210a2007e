"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Sizes run from hand fixtures and brute force on tiny images (all shapes up to 6x6) through
multi-strip images with ragged tails to the full 18 MP, 4096^2 12-bit and 96-image workloads."""
import numpy as np
import pytest

import _pins
import gen
import oracle
from _gpu import assert_result, assert_same, reference, say, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import paper_1707_05062_amd as K
    return K


@pytest.fixture(scope="module")
def ctx(K):
    c = K.Context(0)
    yield c
    c.close()


# ----------------------------------------------------------------------------------------------
# hand fixtures and tiny images

@pytest.mark.parametrize("name", _pins.curve_fixture_names())
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_golden_fixtures(ctx, name, dtype):
    fx = _pins.load_curve_fixture(name)
    img = fx["image"].astype(dtype)
    say("golden", name, dtype.__name__)
    ref = reference(img, fx["M"], fx["nbhd"])
    assert list(ref["sum"]) == list(fx["sum"])
    for src in (img, to_device(img)):
        res = ctx.curve(src, fx["M"], fx["nbhd"])
        assert_result(res, ref, what=name)


def test_tiny_exhaustive(ctx):
    """Every shape up to 6x6, several M, both neighbourhoods, uint8: bit-exact with the oracle."""
    rng = np.random.default_rng(11)
    n = 0
    for H in range(1, 7):
        for W in range(1, 7):
            for M in (1, 2, 3, 5, 8, 16, 33, 256):
                for nbhd in (4, 8):
                    img = rng.integers(0, M, size=(H, W)).astype(np.uint8)
                    res = ctx.curve(img, M, nbhd)
                    assert_result(res, reference(img, M, nbhd), what=f"{H}x{W} M={M} N{nbhd}")
                    n += 1
    say("tiny cases", n)


def test_tiny_u16_large_m(ctx):
    rng = np.random.default_rng(12)
    for H, W in [(1, 1), (1, 5), (5, 1), (3, 4), (6, 6)]:
        for M in (257, 1000, 4096, 10200):
            for nbhd in (4, 8):
                img = rng.integers(0, M, size=(H, W)).astype(np.uint16)
                res = ctx.curve(img, M, nbhd)
                assert_result(res, reference(img, M, nbhd), what=f"u16 {H}x{W} M={M} N{nbhd}")


@pytest.mark.parametrize("block", [256, 512])
def test_large_m_finish_blocks(ctx, K, block):
    """The finishing step for M > 256: each thread takes ceil(M / block) consecutive levels, so the
    last threads get fewer or none (M = 257, 300, 513, 1000, 1025, 3000 against 256 and 512
    threads), with packed and with two-word accumulators, single image and batch."""
    rng = np.random.default_rng(block)
    img0 = gen.random_image(rng, 61, 333, 3000, np.uint16, "smooth")
    for M in (257, 300, 513, 1000, 1025, 3000):
        img = np.minimum(img0, M - 1).astype(np.uint16)
        img[10:20, 40:200] = rng.integers(0, M, size=(10, 160))
        ref = reference(img, M, 4)
        for split in (0, 1):
            ctx.set_plan(2, M, 4, form=K.FORM_MARG, block=block, grid=5, acc_split=split)
            assert_result(ctx.curve(to_device(img), M, 4), ref, what=f"M={M} block {block} split {split}")
        _batch_check(ctx, [img, gen.random_image(rng, 9, 70, M, np.uint16, "uniform")], M, 4)
        ctx.set_plan(2, M, 4)


# ----------------------------------------------------------------------------------------------
# multi-strip images with ragged tails

SHAPES = [(1, 1000), (1000, 1), (37, 301), (64, 257), (5, 2049), (129, 513), (200, 777)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["uniform", "levels", "smooth"])
def test_ragged_u8(ctx, shape, kind):
    rng = np.random.default_rng(hash((shape, kind)) % 2**32)
    for M, nbhd in [(256, 4), (256, 8), (37, 4)]:
        img = gen.random_image(rng, *shape, M, np.uint8, kind)
        res = ctx.curve(to_device(img), M, nbhd)
        assert_result(res, reference(img, M, nbhd), what=f"{shape} {kind} M={M} N{nbhd}")


@pytest.mark.parametrize("shape", [(37, 301), (129, 513), (64, 1100)])
def test_ragged_u16(ctx, shape):
    rng = np.random.default_rng(sum(shape))
    for M, nbhd in [(4096, 4), (4096, 8), (256, 4), (700, 8)]:
        for kind in ("uniform", "smooth"):
            img = gen.random_image(rng, *shape, M, np.uint16, kind)
            res = ctx.curve(to_device(img), M, nbhd)
            assert_result(res, reference(img, M, nbhd), what=f"u16 {shape} {kind} M={M} N{nbhd}")


def test_pitched_and_misaligned(ctx):
    """A column slice of a larger tensor: pitch > W and a base address off the vector alignment."""
    import torch
    rng = np.random.default_rng(5)
    big = gen.random_image(rng, 70, 611, 256, np.uint8, "smooth")
    dev = to_device(big)
    for c0, c1 in [(0, 600), (3, 602), (1, 2), (5, 5 + 256 * 2 + 1)]:
        view = dev[:, c0:c1]
        assert view.stride(0) == 611
        for nbhd in (4, 8):
            res = ctx.curve(view, 256, nbhd)
            assert_result(res, reference(big[:, c0:c1], 256, nbhd), what=f"slice {c0}:{c1} N{nbhd}")
    big16 = gen.random_image(rng, 33, 301, 4096, np.uint16, "smooth")
    dev16 = to_device(big16)
    res = ctx.curve(dev16[:, 1:300], 4096, 8)
    assert_result(res, reference(big16[:, 1:300], 4096, 8), what="u16 slice")
    del torch


# ----------------------------------------------------------------------------------------------
# every launch plan gives the same integers (any partition of the pairs adds up the same)

def test_plan_sweep(ctx, K):
    rng = np.random.default_rng(21)
    img = gen.random_image(rng, 301, 1283, 256, np.uint8, "smooth")
    img[100:140, 200:900] = rng.integers(0, 256, size=(40, 700))  # large gaps: spill path
    dev = to_device(img)
    for nbhd in (4, 8):
        ref = reference(img, 256, nbhd)
        plans = []
        for form, band in [(K.FORM_BAND, 1), (K.FORM_BAND, 2), (K.FORM_BAND, 7), (K.FORM_BAND, 32),
                           (K.FORM_BAND, 64), (K.FORM_MARG, 0), (K.FORM_TRI, 0)]:
            for block in (256, 512):
                for grid in (1, 3, 17, 0):
                    for ppl in (4, 8):
                        plans.append((form, band, block, grid, ppl))
        for form, band, block, grid, ppl in plans:
            for copies in ((1, 2, 4) if form == K.FORM_BAND else (1, 2) if form == K.FORM_MARG else (0,)):
                if copies * (band + 2) * 272 * 4 + 768 * 4 + 512 > 160 * 1024:
                    continue  # the tables would not fit the LDS: the plan is refused
                ctx.set_plan(1, 256, nbhd, form=form, band=band, block=block, grid=grid, px_per_lane=ppl,
                             copies=copies)
                res = ctx.curve(dev, 256, nbhd)
                assert_result(res, ref, what=f"plan {form},{band},{block},{grid},{ppl},c{copies} N{nbhd}")
        say("plans checked", len(plans), "N", nbhd)
    # restore defaults for other tests
    for nbhd in (4, 8):
        ctx.set_plan(1, 256, nbhd)


@pytest.mark.parametrize("W", [512, 520, 1024, 1100, 1536])
def test_packed_strip_borders(ctx, K, W):
    """8-bit pixels, 8 per lane, banded form: strips that end exactly at the right border (the edge
    pixel is the row's own last pixel), strips that cross it, short images (fewer rows than a
    batch or a chunk) and rows with large gaps, over table copies, workgroup sizes and grids, in
    the single-image and the batched launch."""
    rng = np.random.default_rng(W)
    for H in (1, 2, 3, 4, 7, 61):
        img = gen.random_image(rng, H, W, 256, np.uint8, "smooth")
        img[H // 2, W // 3: W // 3 + 200] = rng.integers(0, 256, size=len(img[H // 2, W // 3: W // 3 + 200]))
        dev = to_device(img)
        ref = reference(img, 256, 4)
        for copies in (1, 2, 4):
            for block, grid in [(256, 1), (1024, 3), (1024, 0), (512, 0)]:
                ctx.set_plan(1, 256, 4, form=K.FORM_BAND, band=32, block=block, grid=grid, px_per_lane=8,
                             copies=copies)
                res = ctx.curve(dev, 256, 4)
                assert_result(res, ref, what=f"{H}x{W} c{copies} b{block} g{grid}")
        _batch_check(ctx, [img, gen.random_image(rng, 5, 700, 256, np.uint8, "uniform"), img], 256, 4)
    ctx.set_plan(1, 256, 4)


# ----------------------------------------------------------------------------------------------
# the named workloads at full size

def test_cfg1_exact(ctx):
    img = gen.cfg1_image()
    for nbhd in (4, 8):
        res = ctx.curve(to_device(img), 256, nbhd)
        assert_result(res, reference(img, 256, nbhd), what=f"cfg1 N{nbhd}")


def test_cfg2_full_size_exact(ctx):
    """18 MP u8: every threshold against the brute-force oracle (about 5 s on 8 host cores)."""
    img = gen.cfg2_image()
    say("cfg2 generated", img.shape)
    dev = to_device(img)
    res = ctx.curve(dev, 256, 4)
    say("cfg2 gpu done")
    ref = reference(img, 256, 4)
    say("cfg2 oracle done")
    assert_result(res, ref, what="cfg2 N4")
    # closed forms over the whole curve (independent of the oracle)
    d = _pins.pair_gaps(img, 4)
    assert int(res.count.sum()) == int(d.sum())
    assert int(res.sum.sum()) == int((d * d // 4).sum())


def test_cfg2_async_matches_sync(ctx):
    import torch
    img = gen.cfg2_image()
    dev = to_device(img)
    sync = ctx.curve(dev, 256, 4)
    out = ctx.curve_async(dev, 256, 4)
    out2 = ctx.curve_async(dev, 256, 4)  # a second launch reuses the self-cleaned scratch
    torch.cuda.synchronize()
    for o in (out, out2):
        n, t0, st = [int(x) for x in o["ints"].cpu()]
        assert st == 0
        assert np.array_equal(o["sum"].cpu().numpy(), sync.sum)
        assert np.array_equal(o["count"].cpu().numpy(), sync.count)
        assert np.array_equal(o["C"].cpu().numpy(), sync.C)
        assert list(o["thr"].cpu().numpy()[:n]) == list(sync.thresholds) and t0 == sync.t0


@pytest.mark.parametrize("nbhd", [4, 8])
def test_cfg3_u16_m4096(ctx, nbhd):
    """4096^2 12-bit: full curve against Algorithm 1 (the brute force would take minutes), plus
    eight thresholds against the brute force itself."""
    img = gen.cfg3_image()
    say("cfg3 generated", nbhd)
    res = ctx.curve(to_device(img), 4096, nbhd)
    say("cfg3 gpu done")
    ref = reference(img, 4096, nbhd, exact_all=False)
    assert_result(res, ref, what=f"cfg3 N{nbhd}")
    ts = np.array([0, 1, 700, 1500, 2048, 3000, 4000, 4095], np.int32)
    s, k, c = oracle.curve(img, 4096, nbhd, ts=ts)
    assert np.array_equal(res.sum[ts], s) and np.array_equal(res.count[ts], k)
    assert np.array_equal(res.C[ts], c)


# ----------------------------------------------------------------------------------------------
# two-word accumulators (D1 and E apart), the layout images with 2^30 or more pairs need, forced
# with the plan's acc_split on images of every size

@pytest.fixture
def split_ctx(K):
    c = K.Context(0)
    yield c
    c.close()


def _split(ctx, K, dtype, M, nbhd, **kw):
    ctx.set_plan(dtype, M, nbhd, acc_split=1, **kw)
    assert ctx.get_plan(dtype, 64, 64, M, nbhd)["acc_split"] == 1


def test_split_tiny_and_ragged(split_ctx, K):
    rng = np.random.default_rng(77)
    for M in (1, 2, 5, 37, 256):
        for nbhd in (4, 8):
            _split(split_ctx, K, 1, M, nbhd)
    for H in range(1, 7):
        for W in range(1, 7):
            for M in (2, 5, 256):
                for nbhd in (4, 8):
                    img = rng.integers(0, M, size=(H, W)).astype(np.uint8)
                    assert_result(split_ctx.curve(img, M, nbhd), reference(img, M, nbhd),
                                  what=f"split {H}x{W} M={M} N{nbhd}")
    for shape in SHAPES:
        for M, nbhd in [(256, 4), (256, 8), (37, 4)]:
            img = gen.random_image(rng, *shape, M, np.uint8, "smooth")
            assert_result(split_ctx.curve(to_device(img), M, nbhd), reference(img, M, nbhd),
                          what=f"split {shape} M={M} N{nbhd}")
    for M, nbhd in [(4096, 4), (4096, 8), (700, 8)]:
        _split(split_ctx, K, 2, M, nbhd)
        img = gen.random_image(rng, 129, 513, M, np.uint16, "smooth")
        assert_result(split_ctx.curve(to_device(img), M, nbhd), reference(img, M, nbhd),
                      what=f"split u16 M={M} N{nbhd}")


def test_split_plan_sweep(split_ctx, K):
    rng = np.random.default_rng(78)
    img = gen.random_image(rng, 301, 1283, 256, np.uint8, "smooth")
    img[100:140, 200:900] = rng.integers(0, 256, size=(40, 700))
    dev = to_device(img)
    for nbhd in (4, 8):
        ref = reference(img, 256, nbhd)
        for form, band, copies in [(K.FORM_BAND, 32, 2), (K.FORM_BAND, 7, 4), (K.FORM_MARG, 0, 0),
                                   (K.FORM_TRI, 0, 0)]:
            for block, grid, ppl in [(256, 3, 4), (512, 0, 8), (1024, 0, 8)]:
                if form == K.FORM_MARG and block == 1024:
                    continue  # the marginal instances take at most 512 threads
                if nbhd == 8 and ppl == 8 and block == 1024:
                    continue  # so do the 8-neighbourhood ones with 8 pixels per lane
                _split(split_ctx, K, 1, 256, nbhd, form=form, band=band, block=block, grid=grid,
                       px_per_lane=ppl, copies=copies)
                assert_result(split_ctx.curve(dev, 256, nbhd), ref,
                              what=f"split plan {form},{band},{block},{grid},{ppl} N{nbhd}")


def test_split_cfg2_and_batch(split_ctx, K):
    img = gen.cfg2_image()
    _split(split_ctx, K, 1, 256, 4)
    res = split_ctx.curve(to_device(img), 256, 4)
    d = _pins.pair_gaps(img, 4)
    assert int(res.count.sum()) == int(d.sum()) and int(res.sum.sum()) == int((d * d // 4).sum())
    assert_result(res, reference(img, 256, 4), what="split cfg2")
    rng = np.random.default_rng(79)
    imgs = [gen.random_image(rng, int(rng.integers(1, 200)), int(rng.integers(1, 900)), 256, np.uint8,
                             "smooth") for _ in range(9)]
    _batch_check(split_ctx, imgs, 256, 4)


def test_split_cfg3_n8(split_ctx, K):
    """The M > 256 finishing path with its second gather, on the 4096^2 12-bit workload."""
    img = gen.cfg3_image()
    _split(split_ctx, K, 2, 4096, 8)
    res = split_ctx.curve(to_device(img), 4096, 8)
    assert_result(res, reference(img, 4096, 8, exact_all=False), what="split cfg3 N8")


# ----------------------------------------------------------------------------------------------
# batched launch

def _batch_check(ctx, imgs, M, nbhd, cap=None):
    import torch
    devs = [to_device(im) for im in imgs]
    out = ctx.curve_batch(devs, M, nbhd, capacity=cap)
    torch.cuda.synchronize()
    n = len(imgs)
    ints = out["ints"].cpu().numpy()
    S, Kc, C, T = (out[k].cpu().numpy() for k in ("sum", "count", "C", "thr"))
    for i, im in enumerate(imgs):
        ref = reference(im, M, nbhd, exact_all=im.size <= 300_000)
        assert ints[2 * n + i] == (0 if cap is None or ref["n"] <= cap else -3)
        assert_same(S[i], Kc[i], C[i], T[i], int(ints[n + i]), int(ints[i]), ref,
                    cap=cap, what=f"batch image {i} {im.shape}")
    return out


def test_batch_small_mixed(ctx):
    rng = np.random.default_rng(31)
    imgs = [gen.random_image(rng, int(rng.integers(1, 90)), int(rng.integers(1, 700)), 256, np.uint8,
                             ["uniform", "levels", "smooth"][i % 3]) for i in range(23)]
    for nbhd in (4, 8):
        _batch_check(ctx, imgs, 256, nbhd)


def test_batch_cfg4_full(ctx):
    """The 96-image workload: every image against the oracle, and each image alone == in batch."""
    imgs = gen.batch_images()
    say("cfg4 generated", len(imgs), sum(im.size for im in imgs))
    out = _batch_check(ctx, imgs, 256, 4)
    S = out["sum"].cpu().numpy()
    for i in (0, 17, 95):
        alone = ctx.curve(to_device(imgs[i]), 256, 4)
        assert np.array_equal(alone.sum, S[i])


def test_batch_u16(ctx):
    rng = np.random.default_rng(41)
    imgs = [gen.random_image(rng, int(rng.integers(1, 70)), int(rng.integers(1, 600)), 4096, np.uint16,
                             "smooth") for _ in range(9)]
    _batch_check(ctx, imgs, 4096, 8)


@pytest.mark.parametrize("nbhd", [4, 8])
def test_marginal_copies_u16(ctx, K, nbhd):
    """The marginal form with one and two interleaved table copies (12-bit levels: 2 x 64 KB of
    tables), single image and batch, over workgroup sizes and grids; the copies are summed before
    the merge, so every plan gives the same result."""
    rng = np.random.default_rng(90 + nbhd)
    img = gen.random_image(rng, 129, 1100, 4096, np.uint16, "smooth")
    img[40:60, 100:700] = rng.integers(0, 4096, size=(20, 600))
    dev = to_device(img)
    ref = reference(img, 4096, nbhd)
    for copies in (1, 2):
        for block, grid in [(256, 1), (512, 3), (512, 0)]:
            ctx.set_plan(2, 4096, nbhd, form=K.FORM_MARG, block=block, grid=grid, copies=copies)
            assert_result(ctx.curve(dev, 4096, nbhd), ref, what=f"marg c{copies} b{block} g{grid} N{nbhd}")
        _batch_check(ctx, [img, gen.random_image(rng, 7, 300, 4096, np.uint16, "uniform")], 4096, nbhd)
    with pytest.raises(K.KohlerError):  # four copies of the marginal tables are refused
        ctx.set_plan(2, 4096, nbhd, form=K.FORM_MARG, copies=4)
    ctx.set_plan(2, 4096, nbhd)


# ----------------------------------------------------------------------------------------------
# status codes and scratch hygiene

def test_range_error_and_recovery(ctx, K):
    img = gen.cfg1_image()
    bad = img.copy()
    bad[7, 9] = 200
    res = ctx.curve(to_device(bad), 150, 4, check=False)
    assert res.status == K.E_RANGE
    bad16 = img.astype(np.uint16) * 16
    bad16[100, 200] = 4096
    res = ctx.curve(to_device(bad16), 4096, 8, check=False)
    assert res.status == K.E_RANGE
    # the next call on the same context is unaffected
    ok = np.minimum(img, 149)
    res = ctx.curve(to_device(ok), 150, 4)
    assert_result(res, reference(ok, 150, 4), what="after range error")


def test_capacity(ctx, K):
    img = gen.cfg1_image()
    ref = reference(img, 256, 4)
    assert ref["n"] > 3
    res = ctx.curve(to_device(img), 256, 4, capacity=3)
    assert res.status == K.E_CAPACITY and res.n_thresholds == ref["n"]
    assert list(res.thresholds) == list(ref["thr"][:3])
    assert np.array_equal(res.sum, ref["sum"]) and res.t0 == ref["t0"]
    res = ctx.curve(to_device(img), 256, 4, capacity=0)
    assert res.status == K.E_CAPACITY and len(res.thresholds) == 0


def test_bad_arguments(ctx, K):
    img = to_device(gen.cfg1_image())
    for M, nbhd in [(0, 4), (257, 4), (256, 6), (-1, 8)]:
        with pytest.raises(K.KohlerError) as e:
            ctx.curve(img, M, nbhd)
        assert e.value.status == K.E_ARG
    with pytest.raises(K.KohlerError):
        ctx.curve(img, 256, 4, capacity=-1)


# ----------------------------------------------------------------------------------------------
# the triangular joint histogram (one counter per (lo, hi), no large-gap path) on the same cases

def test_tri_form_cases(K):
    c = K.Context(0)
    try:
        rng = np.random.default_rng(33)
        for dtype in (1, 2):
            for M in (1, 2, 3, 5, 8, 16, 33, 200, 256):
                for nbhd in (4, 8):
                    c.set_plan(dtype, M, nbhd, form=K.FORM_TRI)
        n = 0
        for H in range(1, 7):
            for W in range(1, 7):
                for M in (1, 2, 3, 5, 8, 16, 33, 256):
                    for nbhd in (4, 8):
                        img = rng.integers(0, M, size=(H, W)).astype(np.uint8)
                        assert_result(c.curve(img, M, nbhd), reference(img, M, nbhd), what=f"tri {H}x{W} M={M} N{nbhd}")
                        n += 1
        say("tri tiny cases", n)
        for kind in ("uniform", "levels", "smooth"):
            for (h, w) in [(1, 2000), (257, 1), (77, 515), (130, 1031)]:
                for M, dt in [(256, np.uint8), (200, np.uint8), (256, np.uint16), (33, np.uint16)]:
                    img = gen.random_image(rng, h, w, M, dt, kind)
                    for nbhd in (4, 8):
                        res = c.curve(to_device(img), M, nbhd)
                        assert_result(res, reference(img, M, nbhd), what=f"tri {kind} {h}x{w} M={M} {dt.__name__} N{nbhd}")
        img = gen.cfg1_image()
        for nbhd in (4, 8):
            assert_result(c.curve(to_device(img), 256, nbhd), reference(img, 256, nbhd), what=f"tri cfg1 N{nbhd}")
        # range error under the triangular form, then recovery
        bad = gen.random_image(rng, 50, 90, 200, np.uint8, "smooth")
        bad[10, 10] = 230
        res = c.curve(to_device(bad), 200, 4, check=False)
        assert res.status == K.E_RANGE
        bad[10, 10] = 0
        assert_result(c.curve(to_device(bad), 200, 4), reference(bad, 200, 4), what="tri after range error")
        # batched launch under the triangular form
        imgs = [gen.random_image(rng, h, w, 256, np.uint8, ["uniform", "levels", "smooth"][i % 3])
                for i, (h, w) in enumerate([(1, 1), (3, 700), (129, 257), (600, 41), (255, 1030), (64, 64)])]
        out = c.curve_batch([to_device(x) for x in imgs], 256, 4)
        import torch
        torch.cuda.synchronize()
        ints = out["ints"].cpu().numpy()
        nb = len(imgs)
        for i, x in enumerate(imgs):
            r = reference(x, 256, 4)
            nt = int(ints[i])
            assert_same(out["sum"][i].cpu().numpy(), out["count"][i].cpu().numpy(), out["C"][i].cpu().numpy(),
                        out["thr"][i].cpu().numpy()[:nt], int(ints[nb + i]), nt, r, what=f"tri batch {i}")
    finally:
        c.close()


def test_tri_form_cfg2_full_size(K):
    img = gen.cfg2_image()
    c = K.Context(0)
    try:
        c.set_plan(1, 256, 4, form=K.FORM_TRI)
        res = c.curve(to_device(img), 256, 4)
        assert_result(res, reference(img, 256, 4), what="tri cfg2")
    finally:
        c.close()
