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
