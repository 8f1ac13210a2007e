"""GPU parity of the segmentation by thresholds (class label = number of thresholds below the pixel
value, Sec. 2.1) against the oracle, bit for bit, through the C ABI."""
import numpy as np
import pytest

import gen
import oracle
from _gpu import say, to_device

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


def dev_i32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.int32).reshape(-1) if len(a) else np.zeros(1, np.int32))).cuda()


def labels(ctx, img_dev, thr, M, cap=None, label_dtype=None, n=None):
    import torch
    cap = len(thr) if cap is None else cap
    n_dev = dev_i32([len(thr) if n is None else n])
    out = ctx.segment(img_dev, dev_i32(thr), n_dev, cap, M, label_dtype=label_dtype)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    return res.view(np.uint16) if res.dtype == np.int16 else res


def test_hand_cases(ctx):
    w1 = np.array([[0, 4, 1]], np.uint8)
    assert labels(ctx, to_device(w1), [2], 5).tolist() == [[0, 1, 0]]
    w2 = np.array([[0, 0, 5], [2, 7, 5]], np.uint8)
    assert labels(ctx, to_device(w2), [3], 8).tolist() == [[0, 0, 1], [0, 1, 1]]
    assert labels(ctx, to_device(np.array([[2, 3, 4, 6, 7]], np.uint8)), [3, 6], 8).tolist() == [[0, 0, 1, 1, 2]]
    assert labels(ctx, to_device(np.array([[0, 9, 255]], np.uint8)), [], 256).tolist() == [[0, 0, 0]]


@pytest.mark.parametrize("dtype,M", [(np.uint8, 256), (np.uint8, 37), (np.uint16, 256), (np.uint16, 4096)])
def test_random_shapes(ctx, dtype, M):
    import torch
    rng = np.random.default_rng(M)
    for (h, w) in [(1, 1), (1, 15), (1, 17), (3, 1000), (17, 33), (64, 64), (257, 1031), (1080, 1920)]:
        img = gen.random_image(rng, h, w, M, dtype, ["uniform", "levels", "smooth"][(h + w) % 3])
        k = int(rng.integers(0, min(M, 40)))
        thr = np.sort(rng.choice(M, size=k, replace=False)).astype(np.int32)
        ref = oracle.segment(img, thr)
        for ldt in ([torch.uint8, torch.uint16] if k <= 255 else [torch.uint16]):
            got = labels(ctx, to_device(img), thr, M, label_dtype=ldt)
            assert np.array_equal(got.astype(np.int64), ref), f"{h}x{w} M={M} k={k} {ldt}"
    say("segment random shapes", dtype.__name__, M)


def test_strided_views_and_capacity(ctx):
    import torch
    rng = np.random.default_rng(9)
    img = gen.random_image(rng, 70, 611, 256, np.uint8, "smooth")
    thr = np.array([30, 90, 91, 200], np.int32)
    dev = to_device(img)
    view = dev[:, 3:600]
    got = labels(ctx, view, thr, 256)
    assert np.array_equal(got.astype(np.int64), oracle.segment(img[:, 3:600], thr))
    # an output with a pitch
    big = torch.zeros((70, 700), dtype=torch.uint8, device=dev.device)
    out = ctx.segment(dev, dev_i32(thr), dev_i32([4]), 4, 256, out=big[:, 5:616])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.int64), oracle.segment(img, thr))
    assert int(big[:, :5].abs().sum()) == 0 and int(big[:, 616:].abs().sum()) == 0
    # a count above the capacity uses the first `capacity` thresholds
    got = labels(ctx, dev, thr, 256, cap=2, n=4)
    assert np.array_equal(got.astype(np.int64), oracle.segment(img, thr[:2]))


def test_after_the_curve(ctx, K):
    """The whole path on the 18 MP image: curve, thresholds and labels stay on the device."""
    import torch
    img = gen.cfg2_image()
    dev = to_device(img)
    out = ctx.curve_async(dev, 256, 4, capacity=128)
    lab = ctx.segment(dev, out["thr"], out["ints"][0:1], 128, 256)
    torch.cuda.synchronize()
    n = int(out["ints"][0])
    thr = out["thr"].cpu().numpy()[:n]
    ref_thr, _, _, _ = oracle.thresholds(*oracle.alg1(img, 256, 4))
    assert list(thr) == list(ref_thr)
    assert np.array_equal(lab.cpu().numpy().astype(np.int64), oracle.segment(img, ref_thr))
    say("segment 18 MP", n, "thresholds")


def test_bad_arguments(ctx, K):
    import torch
    dev = to_device(np.zeros((4, 4), np.uint8))
    thr = dev_i32([1, 2])
    n = dev_i32([2])
    with pytest.raises(K.KohlerError):
        ctx.segment(dev, thr, n, 300, 256)  # capacity above M
    with pytest.raises(K.KohlerError):
        ctx.segment(dev, thr, n, 2, 0)      # M below 1
    with pytest.raises(K.KohlerError):
        ctx.segment(dev, thr, n, 256, 256, label_dtype=torch.uint8)  # labels up to 256 need u16


def test_values_at_or_above_M(ctx):
    """A value >= M lies above every threshold (t < M), also when the last threshold is M - 1."""
    import torch
    rng = np.random.default_rng(21)
    img = rng.integers(0, 100, size=(37, 301)).astype(np.uint16)
    thr = np.array([3, 17, 39], np.int32)  # M = 40: t_k = M - 1
    got = labels(ctx, to_device(img), thr, 40, label_dtype=torch.uint8)
    assert np.array_equal(got.astype(np.int64), oracle.segment(img, thr))


def _stats(ctx, img, thr, M, cap=None):
    import torch
    cap = len(thr) if cap is None else cap
    dev = to_device(img)
    c, s, m = ctx.class_stats(dev, dev_i32(thr), dev_i32([len(thr)]), cap, M)
    torch.cuda.synchronize()
    return c.cpu().numpy(), s.cpu().numpy(), m.cpu().numpy()


@pytest.mark.parametrize("dtype,M", [(np.uint8, 256), (np.uint8, 37), (np.uint16, 4096), (np.uint16, 10200)])
def test_class_stats_and_mean_image(ctx, dtype, M):
    import torch
    rng = np.random.default_rng(100 + M)
    for (h, w) in [(1, 1), (1, 17), (3, 1000), (17, 33), (257, 1031), (1080, 1920)]:
        img = gen.random_image(rng, h, w, M, dtype, ["uniform", "levels", "smooth"][(h + w) % 3])
        k = int(rng.integers(0, min(M, 40)))
        thr = np.sort(rng.choice(M, size=k, replace=False)).astype(np.int32)
        rc, rs, rm = oracle.class_stats(img, thr, M)
        c, s, m = _stats(ctx, img, thr, M)
        assert np.array_equal(c, rc) and np.array_equal(s, rs), f"{h}x{w} M={M} k={k}"
        assert np.array_equal(m.view(np.int64), rm.view(np.int64)), f"{h}x{w} M={M} k={k}"  # same bits
        dev = to_device(img)
        out = ctx.mean_image(dev, dev_i32(thr), dev_i32([k]), k, M, torch.from_numpy(rm).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(img.dtype) if out.dtype != torch.uint8 else out.cpu().numpy(),
                              oracle.mean_image(img, thr, M)), f"{h}x{w} M={M} k={k}"
    say("class stats", dtype.__name__, M)


def test_class_stats_capacity_and_repeat(ctx):
    """Entries past the classes in use are 0; the scratch histogram is clear for the next call."""
    rng = np.random.default_rng(31)
    big = gen.random_image(rng, 700, 900, 256, np.uint8, "smooth")
    small = gen.random_image(rng, 33, 65, 256, np.uint8, "uniform")
    thr = np.array([40, 90, 200], np.int32)
    for img in (big, small, big):
        c, s, m = _stats(ctx, img, thr, 256, cap=6)
        rc, rs, rm = oracle.class_stats(img, thr, 256)
        assert np.array_equal(c[:4], rc) and np.array_equal(s[:4], rs) and np.array_equal(m[:4], rm)
        assert not c[4:].any() and not s[4:].any() and not m[4:].any()
    # values >= M count in the top class at the value M
    img = rng.integers(0, 100, size=(20, 50)).astype(np.uint16)
    c, s, m = _stats(ctx, img, np.array([5, 39], np.int32), 40)
    rc, rs, rm = oracle.class_stats(img, [5, 39], 40)
    assert np.array_equal(c, rc) and np.array_equal(s, rs) and np.array_equal(m, rm)


def test_top_thresholds(ctx):
    import torch
    rng = np.random.default_rng(41)
    for trial in range(30):
        M = int(rng.integers(2, 600))
        cnt = rng.integers(0, 50, size=M).astype(np.int64)
        sm = (cnt * rng.integers(0, 4, size=M)).astype(np.int64)  # many equal C values
        if trial % 3 == 0:
            sm = rng.integers(0, 2 ** 40, size=M).astype(np.int64)
            cnt = rng.integers(1, 2 ** 20, size=M).astype(np.int64)
        n = int(rng.integers(0, min(M, 300) + 1))
        thr = np.sort(rng.choice(M, size=n, replace=False)).astype(np.int32)
        k = int(rng.integers(0, n + 3))
        top, n_top = ctx.top_thresholds(torch.from_numpy(sm).cuda(), torch.from_numpy(cnt).cuda(), dev_i32(thr),
                                        dev_i32([n]), max(n, 1), M, k)
        torch.cuda.synchronize()
        want = oracle.top_thresholds(sm, cnt, thr, k)
        assert int(n_top[0]) == len(want)
        assert top.cpu().numpy()[:len(want)].tolist() == want, (trial, M, n, k)
    # the doubles of 2^53 and 2^53 + 1 are equal; the exact order is not
    sm = torch.tensor([2 ** 53, 2 ** 53 + 1], dtype=torch.int64).cuda()
    one = torch.ones(2, dtype=torch.int64).cuda()
    top, n_top = ctx.top_thresholds(sm, one, dev_i32([0, 1]), dev_i32([2]), 2, 2, 1)
    torch.cuda.synchronize()
    assert top.cpu().tolist()[:1] == [1] and int(n_top[0]) == 1


def test_whole_path_18mp(ctx, K):
    """Curve, thresholds, the 6 most significant, their class statistics and the class-mean image,
    all on the device, for the 18 MP image."""
    import torch
    img = gen.cfg2_image()
    dev = to_device(img)
    out = ctx.curve_async(dev, 256, 4, capacity=128)
    top, n_top = ctx.top_thresholds(out["sum"], out["count"], out["thr"], out["ints"][0:1], 128, 256, 6)
    top_sorted, _ = torch.sort(top[:6])
    c, s, m = ctx.class_stats(dev, top_sorted, n_top, 6, 256)
    mi = ctx.mean_image(dev, top_sorted, n_top, 6, 256, m)
    torch.cuda.synchronize()
    ref_s, ref_k = oracle.alg1(img, 256, 4)
    ref_thr, _, _, _ = oracle.thresholds(ref_s, ref_k)
    want = oracle.top_thresholds(ref_s, ref_k, ref_thr, 6)
    assert int(n_top[0]) == len(want) and top.cpu().numpy()[:len(want)].tolist() == want
    sel = sorted(want)
    rc, rsum, rm = oracle.class_stats(img, sel, 256)
    n = len(sel)
    assert np.array_equal(c.cpu().numpy()[:n + 1], rc) and np.array_equal(s.cpu().numpy()[:n + 1], rsum)
    assert np.array_equal(m.cpu().numpy()[:n + 1], rm)
    assert np.array_equal(mi.cpu().numpy(), oracle.mean_image(img, sel, 256))
    say("18 MP: the 6 most significant thresholds", sel, "class means", np.round(rm, 2).tolist())


def test_consumer_bad_arguments(ctx, K):
    import torch
    dev = to_device(np.zeros((4, 4), np.uint8))
    thr, n = dev_i32([1, 2]), dev_i32([2])
    with pytest.raises(K.KohlerError):
        ctx.class_stats(dev, thr, n, 257, 256)   # capacity above M
    with pytest.raises(K.KohlerError):
        ctx.mean_image(dev, thr, n, 2, 256, None)  # no class means
    s = torch.zeros(256, dtype=torch.int64).cuda()
    with pytest.raises(K.KohlerError):
        ctx.top_thresholds(s, s, thr, n, 2, 256, -1)  # negative k
