"""Synthetic workloads standing in for the paper's images and video.

The paper measures on two photographs (512x512 "Lenna", 3672x4896 "Tulips", Sec. 4 Table 1) and on a
502x480 video clip from YFCC100M (Sec. 4 Table 2). None of them is available, so seeded synthetic
images of the same kind stand in: piecewise-smooth scenes with sharp region boundaries plus sensor
noise, which is what a contrast-thresholding method is meant to segment.

Every generator uses numpy's PCG64 with an explicit seed, synthesises in float64, rounds with
``np.rint`` (half to even) and clips to [0, M-1] before the integer cast.

Named workloads:
  cfg1  256x256 u8, M=256: 2x3 grid of rectangles, means U(20,235), noise N(0, 8^2).
  cfg2  3456x5184 u8 (about 18 MP, the size of the paper's largest photograph), M=256: smooth
        cosine background (amplitude 60) plus 40 painted ellipses with means U(0,255),
        noise N(0, 5^2).
  cfg3  4096x4096 u16 with 12-bit values, M=4096: 500-site Voronoi cells with values U{0..4095},
        noise N(0, 30^2).
  cfg4  96 u8 images, sizes log-uniform between 128x128 and 4000x3000, aspect ratio in
        {1, 4/3, 16/9}, cfg1-style content with the grid scaled.
  cfg5  a served mix: 1920x1080 video frames (a 40-blob canvas seen through a window that moves
        2 px per frame, fresh N(0, 6^2) noise per frame), 3840x2160 frames built the same way,
        and cfg2-style 18 MP stills.
"""
from __future__ import annotations

import math

import numpy as np

CONFIGS = {
    "cfg1": dict(H=256, W=256, dtype="u8", M=256, seed=1),
    "cfg2": dict(H=3456, W=5184, dtype="u8", M=256, seed=2),
    "cfg3": dict(H=4096, W=4096, dtype="u16", M=4096, seed=3),
    "cfg4": dict(n=96, dtype="u8", M=256, seed=4),
    "cfg5": dict(rate=240.0, dtype="u8", M=256, seed=5),
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _finish(x: np.ndarray, M: int, dtype) -> np.ndarray:
    return np.clip(np.rint(x), 0, M - 1).astype(dtype)


def _grid_rectangles(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    """2x3 grid of constant rectangles; cut positions scale with the image (cfg1 uses 256x256)."""
    r_lo, r_hi = (H * 64) // 256, (H * 192) // 256
    c_lo, c_hi = (W * 32) // 256, (W * 224) // 256
    gap = max(1, (W * 32) // 256)
    row_cut = int(rng.integers(r_lo, r_hi + 1))
    while True:
        cols = np.sort(rng.integers(c_lo, c_hi + 1, size=2))
        if cols[1] - cols[0] >= gap:
            break
    means = rng.uniform(20.0, 235.0, size=(2, 3))
    img = np.empty((H, W), dtype=np.float64)
    rows = [(0, row_cut), (row_cut, H)]
    colr = [(0, int(cols[0])), (int(cols[0]), int(cols[1])), (int(cols[1]), W)]
    for i, (r0, r1) in enumerate(rows):
        for j, (c0, c1) in enumerate(colr):
            img[r0:r1, c0:c1] = means[i, j]
    return img


def cfg1_image(seed: int = 1, H: int = 256, W: int = 256, sigma: float = 8.0) -> np.ndarray:
    """cfg1: six rectangular regions with constant means plus Gaussian noise, u8."""
    rng = _rng(seed)
    img = _grid_rectangles(rng, H, W)
    img += rng.normal(0.0, sigma, size=(H, W))
    return _finish(img, 256, np.uint8)


def _paint_ellipses(rng: np.random.Generator, img: np.ndarray, n: int, scale: float) -> None:
    H, W = img.shape
    for _ in range(n):
        cy = rng.uniform(0.0, H)
        cx = rng.uniform(0.0, W)
        ay = rng.uniform(0.01, 0.08) * scale
        ax = rng.uniform(0.01, 0.08) * scale
        th = rng.uniform(0.0, math.pi)
        mean = rng.uniform(0.0, 255.0)
        r = max(ax, ay)
        y0, y1 = max(0, int(cy - r) - 1), min(H, int(cy + r) + 2)
        x0, x1 = max(0, int(cx - r) - 1), min(W, int(cx + r) + 2)
        if y0 >= y1 or x0 >= x1:
            continue
        yy = np.arange(y0, y1, dtype=np.float64)[:, None] + 0.5 - cy
        xx = np.arange(x0, x1, dtype=np.float64)[None, :] + 0.5 - cx
        c, s = math.cos(th), math.sin(th)
        u = xx * c + yy * s
        v = -xx * s + yy * c
        inside = (u / ax) ** 2 + (v / ay) ** 2 <= 1.0
        img[y0:y1, x0:x1][inside] = mean


def blob_canvas(seed: int, H: int, W: int, n_blobs: int = 40, scale: float | None = None) -> np.ndarray:
    """Noise-free float64 scene: cosine background (amplitude 60 around 128) plus painted ellipses."""
    rng = _rng(seed)
    kx, ky = rng.integers(1, 4, size=2)
    px, py = rng.uniform(0.0, 1.0, size=2)
    x = np.arange(W, dtype=np.float64)
    y = np.arange(H, dtype=np.float64)
    bx = np.cos(2.0 * math.pi * (kx * x / W + px))
    by = np.cos(2.0 * math.pi * (ky * y / H + py))
    img = 128.0 + 60.0 * by[:, None] * bx[None, :]
    _paint_ellipses(rng, img, n_blobs, float(min(H, W)) if scale is None else scale)
    return img


def cfg2_image(seed: int = 2, H: int = 3456, W: int = 5184, sigma: float = 5.0) -> np.ndarray:
    """cfg2: about 18 MP u8 scene, cosine background plus 40 ellipses plus N(0, 5^2) noise."""
    img = blob_canvas(seed, H, W)
    img += _rng(seed + 1_000_000).normal(0.0, sigma, size=(H, W))
    return _finish(img, 256, np.uint8)


def cfg3_image(seed: int = 3, H: int = 4096, W: int = 4096, sites: int = 500,
               M: int = 4096, sigma: float = 30.0) -> np.ndarray:
    """cfg3: Voronoi cells with values U{0..M-1} plus N(0, 30^2) noise, u16 holding 12-bit values."""
    from scipy.spatial import cKDTree

    rng = _rng(seed)
    pts = np.column_stack([rng.uniform(0.0, H, size=sites), rng.uniform(0.0, W, size=sites)])
    vals = rng.integers(0, M, size=sites).astype(np.float64)
    tree = cKDTree(pts)
    img = np.empty((H, W), dtype=np.float64)
    xs = np.arange(W, dtype=np.float64) + 0.5
    step = 256
    for r0 in range(0, H, step):
        r1 = min(H, r0 + step)
        ys = np.arange(r0, r1, dtype=np.float64) + 0.5
        q = np.column_stack([np.repeat(ys, W), np.tile(xs, r1 - r0)])
        _, idx = tree.query(q)
        img[r0:r1] = vals[idx].reshape(r1 - r0, W)
    img += rng.normal(0.0, sigma, size=(H, W))
    return _finish(img, M, np.uint16)


def batch_sizes(seed: int = 4, n: int = 96) -> list[tuple[int, int]]:
    """cfg4 image shapes: pixel count log-uniform in [128^2, 4000*3000], aspect in {1, 4/3, 16/9}."""
    rng = _rng(seed)
    out = []
    aspects = [1.0, 4.0 / 3.0, 16.0 / 9.0]
    for _ in range(n):
        npx = math.exp(rng.uniform(math.log(128 * 128), math.log(4000 * 3000)))
        r = aspects[int(rng.integers(0, 3))]
        W = int(round(math.sqrt(npx * r)))
        H = int(round(W / r))
        W = min(max(W, 128), 4000)
        H = min(max(H, 128), 3000)
        out.append((H, W))
    return out


def batch_images(seed: int = 4, n: int = 96, max_images: int | None = None) -> list[np.ndarray]:
    """cfg4: n u8 images of uneven sizes; image i draws its content from seed 4000+i."""
    shapes = batch_sizes(seed, n)
    if max_images is not None:
        shapes = shapes[:max_images]
    return [cfg1_image(seed * 1000 + i, H, W) for i, (H, W) in enumerate(shapes)]


def serve_pool(seed: int = 5, n1080: int = 64, n4k: int = 16, n18: int = 4) -> dict[str, list[np.ndarray]]:
    """cfg5 frame pool: moving-window 1080p and 4K frames plus 18 MP stills (cycled by the server bench)."""
    rng = _rng(seed)
    out: dict[str, list[np.ndarray]] = {}
    for name, (H, W, nf, cseed) in {"1080p": (1080, 1920, n1080, seed * 10 + 1),
                                    "4k": (2160, 3840, n4k, seed * 10 + 2)}.items():
        canvas = blob_canvas(cseed, H, W + 2 * nf, scale=float(H))
        frames = []
        for k in range(nf):
            win = canvas[:, 2 * k: 2 * k + W] + rng.normal(0.0, 6.0, size=(H, W))
            frames.append(_finish(win, 256, np.uint8))
        out[name] = frames
    out["18mp"] = [cfg2_image(seed * 1000 + 100 + j) for j in range(n18)]
    return out


def random_image(rng: np.random.Generator, H: int, W: int, M: int, dtype=np.uint8,
                 kind: str = "uniform") -> np.ndarray:
    """Small test images: uniform values, a few flat levels, or a smooth ramp plus noise."""
    if kind == "uniform":
        return rng.integers(0, M, size=(H, W)).astype(dtype)
    if kind == "levels":
        lv = rng.integers(0, M, size=max(1, min(M, 4)))
        return lv[rng.integers(0, len(lv), size=(H, W))].astype(dtype)
    if kind == "smooth":
        y = np.arange(H, dtype=np.float64)[:, None]
        x = np.arange(W, dtype=np.float64)[None, :]
        base = (M - 1) * (0.5 + 0.4 * np.sin(0.05 * x + 0.03 * y + rng.uniform(0, 6.28)))
        return _finish(base + rng.normal(0.0, max(1.0, M / 64.0), size=(H, W)), M, dtype)
    raise ValueError(kind)


def two_level_image(rng: np.random.Generator, H: int, W: int, a: int, b: int, dtype=np.uint8) -> np.ndarray:
    """Random two-level image with values in {a, b}."""
    return np.where(rng.integers(0, 2, size=(H, W)) == 1, b, a).astype(dtype)
