"""GPU tests of the serving loop and the autotuner, through the C ABI.

Every request's result must be the same whether it ran alone (a graph replay), in a batch with
others (one persistent launch), or through the plain context call, and equal to the oracle where the
oracle is cheap: images are independent (Sec. 2.1), so membership in a launch cannot change a
result."""
import numpy as np
import pytest

import gen
from _gpu import assert_result, assert_same, reference, say, to_device

pytestmark = pytest.mark.gpu

M = 256


@pytest.fixture(scope="module")
def K():
    import paper_1707_05062_amd as K
    return K


@pytest.fixture(scope="module")
def ctx(K):
    c = K.Context(0)
    yield c
    c.close()


def mixed_images():
    """Mixed shapes (ragged strips, single rows and columns, a 1080p frame) and contents."""
    rng = np.random.default_rng(77)
    shapes = [(256, 256), (1, 700), (333, 1), (97, 515), (480, 640), (1080, 1920), (257, 1031), (64, 64)]
    out = []
    for i, (h, w) in enumerate(shapes):
        if i % 3 == 0:
            img = gen.random_image(np.random.default_rng(500 + i), h, w, M, np.uint8, "smooth")
        elif i % 3 == 1:
            img = rng.integers(0, M, size=(h, w)).astype(np.uint8)
        else:
            img = gen.random_image(np.random.default_rng(500 + i), h, w, M, np.uint8, "levels")
        out.append(np.ascontiguousarray(img.astype(np.uint8)))
    return out


def as_kind(img, kind):
    import torch
    if kind == "pageable":
        return img
    t = torch.from_numpy(img)
    return t.pin_memory() if kind == "pinned" else t.cuda()


def same(a, b, what):
    assert np.array_equal(a.sum, b.sum), what
    assert np.array_equal(a.count, b.count), what
    assert np.array_equal(a.C, b.C), what
    assert a.n_thresholds == b.n_thresholds and a.t0 == b.t0, what
    assert list(a.thresholds) == list(b.thresholds), what


def test_alone_and_in_the_mix(K, ctx):
    imgs = mixed_images()
    kinds = ["pinned", "pageable", "device"]
    plain = [ctx.curve(im, M, 4) for im in imgs]
    for i in (0, 1, 2, 3, 7):  # oracle on the cheap ones
        assert_result(plain[i], reference(imgs[i], M, 4), what=f"plain {imgs[i].shape}")
    srv = K.Server(ctx, M=M, nbhd=4, slots=8, lanes=2, max_batch=8, hbm_budget_bytes=256 << 20, use_graphs=True)
    try:
        # alone: one request at a time (graph replays)
        alone = []
        for i, im in enumerate(imgs):
            src = as_kind(im, kinds[i % 3])
            res, info = srv.wait(srv.submit(src))
            assert info["batch"] == 1 and info["graph"] == 1, info
            alone.append(res)
        # in the mix: everything admitted together (batched launches), twice
        for rnd in range(2):
            srcs = [as_kind(im, kinds[(i + rnd) % 3]) for i, im in enumerate(imgs)]
            srv.pause(True)
            tickets = [srv.submit(s) for s in srcs]
            srv.pause(False)
            mixed = [srv.wait(t) for t in tickets]
            assert max(info["batch"] for _, info in mixed) > 1
            for i, (res, info) in enumerate(mixed):
                what = f"round {rnd} image {i} {imgs[i].shape} batch {info['batch']}"
                same(res, plain[i], what)
                same(alone[i], plain[i], what + " alone")
        st = srv.stats()
        say("server stats", st)
        assert st["graph_launches"] >= len(imgs) and st["batched_launches"] >= 2
        assert st["completed"] == 3 * len(imgs) and st["peak_inflight"] <= 8
    finally:
        srv.close()


def test_graph_replays_with_eager_work_between(K, ctx):
    """One shape replayed many times with different contents, eager context calls in between:
    every replay must equal the eager result of the same image."""
    srv = K.Server(ctx, M=M, nbhd=4, slots=2, lanes=1, max_batch=1, hbm_budget_bytes=64 << 20, use_graphs=True)
    try:
        for k in range(6):
            img = gen.random_image(np.random.default_rng(900 + k), 300, 700, M, np.uint8, "smooth" if k % 2 else "uniform").astype(np.uint8)
            eager = ctx.curve(to_device(img), M, 4)
            res, info = srv.wait(srv.submit(as_kind(img, "pinned")))
            assert info["graph"] == 1
            same(res, eager, f"replay {k}")
        st = srv.stats()
        assert st["graphs_built"] == 1 and st["graph_launches"] == 6, st
    finally:
        srv.close()


def test_hbm_budget_admission_and_refusals(K, ctx):
    img = gen.random_image(np.random.default_rng(31), 512, 1024, M, np.uint8, "smooth").astype(np.uint8)
    probe = K.Server(ctx, M=M, slots=8, lanes=2, max_batch=8, queue_capacity=6, hbm_budget_bytes=64 << 20)
    slot_state = probe.stats()["slot_state_bytes"]
    probe.close()
    # room for two images at a time
    budget = slot_state + 2 * img.nbytes + 1024
    srv = K.Server(ctx, M=M, slots=8, lanes=2, max_batch=8, queue_capacity=6, hbm_budget_bytes=budget)
    try:
        ref = ctx.curve(img, M, 4)
        big = np.zeros((1024, 2048), np.uint8)  # larger than the whole arena
        with pytest.raises(K.KohlerError) as e:
            srv.submit(big)
        assert e.value.status == K.E_BUSY
        srv.pause(True)
        src = as_kind(img, "pinned")
        tickets = [srv.submit(src) for _ in range(6)]
        with pytest.raises(K.KohlerError) as e:
            srv.submit(src)  # queue full
        assert e.value.status == K.E_BUSY
        assert srv.cancel(tickets[-1])
        srv.pause(False)
        for t in tickets[:-1]:
            res, info = srv.wait(t)
            same(res, ref, "budget")
            assert info["batch"] <= 2
        res, info = srv.wait(tickets[-1])
        assert res.status == K.E_CANCELED
        st = srv.stats()
        say("budget stats", st)
        assert st["peak_inflight"] <= 2 and st["arena_peak_bytes"] <= st["arena_bytes"]
        assert st["refused"] == 2 and st["cancelled"] == 1
    finally:
        srv.close()


def test_request_status_is_per_request(K, ctx):
    """A pixel >= M fails only its own request, also inside a batch."""
    Ms = 200
    good = gen.random_image(np.random.default_rng(41), 200, 300, Ms, np.uint8, "smooth").astype(np.uint8)
    bad = good.copy()
    bad[100, 150] = 250
    srv = K.Server(ctx, M=Ms, slots=4, lanes=1, max_batch=4, hbm_budget_bytes=64 << 20)
    try:
        ref = reference(good, Ms, 4)
        srv.pause(True)
        tickets = [srv.submit(x) for x in (good, bad, good)]
        srv.pause(False)
        out = [srv.wait(t) for t in tickets]
        assert out[1][0].status == K.E_RANGE
        for res, _ in (out[0], out[2]):
            assert_result(res, ref, what="good in batch with a bad image")
        res, _ = srv.wait(srv.submit(bad))
        assert res.status == K.E_RANGE
        res, _ = srv.wait(srv.submit(good))
        assert_result(res, ref, what="good after a bad image")
    finally:
        srv.close()


def test_autotune_keeps_results(K, ctx):
    img = gen.cfg1_image()
    dev = to_device(img)
    ref = reference(img, M, 4)
    c2 = K.Context(0)
    try:
        plan, us = c2.autotune([dev], M, 4, reps=3)
        say("tuned single", plan, us)
        assert plan["block"] in (256, 512) and plan["px_per_lane"] in (4, 8) and us > 0
        assert_result(c2.curve(dev, M, 4), ref, what="after single-image tuning")
        batch = [to_device(gen.random_image(np.random.default_rng(60 + h), h, w, M, np.uint8, "smooth").astype(np.uint8))
                 for h, w in [(128, 128), (300, 500), (777, 333), (1000, 1500)]]
        plan_b, us_b = c2.autotune(batch, M, 4, reps=3)
        say("tuned batch", plan_b, us_b)
        out = c2.curve_batch(batch, M, 4)
        import torch
        torch.cuda.synchronize()
        n = len(batch)
        ints = out["ints"].cpu().numpy()
        for i, im in enumerate(batch):
            r = reference(im.cpu().numpy(), M, 4)
            nt = int(ints[i])
            assert_same(out["sum"][i].cpu().numpy(), out["count"][i].cpu().numpy(), out["C"][i].cpu().numpy(),
                        out["thr"][i].cpu().numpy()[:nt], int(ints[n + i]), nt, r, what=f"batch tuned {i}")
            assert int(ints[2 * n + i]) == 0
    finally:
        c2.close()


def test_tuned_plan_cache(K, ctx, tmp_path):
    from paper_1707_05062_amd import tuning
    dev = to_device(gen.cfg1_image())
    c2 = K.Context(0)
    try:
        path = str(tmp_path / "plans.json")
        p1, us1, hit1 = tuning.tuned_plan(c2, [dev], M, 4, path=path, reps=3)
        p2, us2, hit2 = tuning.tuned_plan(c2, [dev], M, 4, path=path)
        assert not hit1 and hit2 and p1 == p2 and us1 == us2
    finally:
        c2.close()


# ----------------------------------------------------------------------------------------------
# video mode: each frame segmented in two classes at its own t0 (eq (4); Sec. 4's video experiment)

def two_class(img, t0):
    """The oracle's labels at one threshold (class = number of thresholds below the value), one
    class when the curve is identically zero (t0 = -1)."""
    import oracle
    return oracle.segment(img, [t0] if t0 >= 0 else []).astype(np.uint8)


def label_buffer(H, W, kind, wide=0):
    import torch
    if kind == "pageable":
        return np.full((H, W + wide), 7, np.uint8)[:, :W]
    t = torch.full((H, W + wide), 7, dtype=torch.uint8)
    t = t.pin_memory() if kind == "pinned" else t.cuda()
    return t[:, :W]


def labels_np(buf):
    import torch
    return buf.cpu().numpy() if isinstance(buf, torch.Tensor) else np.asarray(buf)


def video_frames():
    pool = gen.serve_pool(n1080=4, n4k=0, n18=0)
    frames = list(pool["1080p"]) + mixed_images()[:6]
    frames.append(np.full((40, 70), 9, np.uint8))  # constant: C identically zero, t0 = -1
    return frames


def test_video_t0_labels_alone_and_in_the_mix(K, ctx):
    import torch
    frames = video_frames()
    refs = [reference(f, M, 4, exact_all=f.size <= 3_000_000) for f in frames]
    want = [two_class(f, r["t0"]) for f, r in zip(frames, refs)]
    assert refs[-1]["t0"] == -1 and not want[-1].any()
    img_kinds = ["pinned", "pageable", "device"]
    lab_kinds = ["device", "pinned", "pageable"]
    for cfg in (dict(slots=1, lanes=1, max_batch=1), dict(slots=8, lanes=2, max_batch=8)):
        srv = K.Server(ctx, M=M, nbhd=4, hbm_budget_bytes=256 << 20, label_t0=True, **cfg)
        try:
            for rnd in range(2):
                bufs = [label_buffer(*f.shape, lab_kinds[(i + rnd) % 3], wide=3 * (i % 2)) for i, f in enumerate(frames)]
                srcs = [as_kind(f, img_kinds[(i + rnd) % 3]) for i, f in enumerate(frames)]
                if cfg["max_batch"] > 1:
                    srv.pause(True)
                tickets = [srv.submit(src, labels=b) for src, b in zip(srcs, bufs)]
                if cfg["max_batch"] > 1:
                    srv.pause(False)
                results = [srv.wait(t) for t in tickets]
                torch.cuda.synchronize()
                if cfg["max_batch"] > 1:
                    assert max(info["batch"] for _, info in results) > 1
                for i, ((res, info), b) in enumerate(zip(results, bufs)):
                    what = f"{cfg} round {rnd} frame {i} {frames[i].shape} labels {lab_kinds[(i + rnd) % 3]}"
                    assert_result(res, refs[i], what=what)
                    assert info["graph"] == 0
                    got = labels_np(b)
                    assert np.array_equal(got, want[i]), what
            say("video mode", cfg, srv.stats())
        finally:
            srv.close()


def test_video_mode_requires_label_t0(K, ctx):
    srv = K.Server(ctx, M=M, nbhd=4, slots=2, lanes=1, max_batch=1, hbm_budget_bytes=64 << 20)
    try:
        f = np.zeros((8, 8), np.uint8)
        with pytest.raises(K.KohlerError):
            srv.submit(f, labels=np.zeros((8, 8), np.uint8))
        res, _ = srv.wait(srv.submit(f))  # the server still serves curves
        assert res.t0 == -1
    finally:
        srv.close()
