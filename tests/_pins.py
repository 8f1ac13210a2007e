"""Pins for the CPU oracle: checks that tie it to the paper and to mathematics, not to itself.

Each ``pin_*`` function takes an oracle library handle (``None`` = the committed oracle) and raises
AssertionError on a mismatch. The same functions run against deliberately broken builds of the
oracle in ``test_oracle_mutants.py`` to show that each plausible mistake is caught.

Sources of truth (G. Noyel, arXiv 1707.05062):
  - hand-worked examples from the definitions of Sec. 2.1, eqs (1)-(4)  (tests/golden/*.txt);
  - closed forms: over thresholds, sum_t #B(t) = sum over unordered pairs of |f(p) - f(q)|, and
    sum_t sum(t) = sum over pairs of floor(d^2 / 4), because for a gap d the contrasts
    min(d - u, u) for u = 0..d-1 add up to floor(d^2 / 4);
  - special cases with a closed form (constant image, two-level image, unit ramp);
  - exact symmetries (transpose, flips, grey-level inversion, grey-level shift);
  - bounds (0 <= C(t) <= min(t, M-1-t), #B(M-1) = 0);
  - the half-neighbourhood theorem of Sec. 3.2 (eq (9)) via Algorithm 1 (Sec. 3.1);
  - the direct route of Sec. 3.1: boundary pixels as the dilation of C_1^t minus C_1^t;
  - for other neighbourhoods (a symmetric structuring element, the hexagonal 6-neighbourhood):
    hand-worked examples, eq (9) through Algorithm 1, the same closed forms over an independently
    enumerated pair list, the direct route, and reductions to N4/N8 (the offset sets of N4 and N8,
    and the hexagonal grid on one row or one column, which has only N4's pairs);
  - for the 3x3 binomial pre-filter: hand-worked values, constant images, the impulse response,
    the separable route, transposition and the value range.
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ----------------------------------------------------------------------------------------------
# golden fixtures

def _parse_line(line: str):
    key, _, rest = line.partition(" ")
    return key, rest.split()


def load_curve_fixture(name: str) -> dict:
    d: dict = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = _parse_line(line)
            d[k] = v
    H, W = int(d["H"][0]), int(d["W"][0])
    return dict(
        image=np.array([int(x) for x in d["image"]], dtype=np.int64).reshape(H, W),
        M=int(d["M"][0]), nbhd=int(d["nbhd"][0]),
        sum=np.array([int(x) for x in d["sum"]], np.int64),
        count=np.array([int(x) for x in d["count"]], np.int64),
        C=[Fraction(x) for x in d["C"]],
        thresholds=[int(x) for x in d.get("thresholds", [])],
        t0=int(d["t0"][0]),
    )


def curve_fixture_names() -> list[str]:
    return sorted(f for f in os.listdir(GOLDEN) if f.startswith("w") and f.endswith(".txt"))


def load_threshold_cases() -> list[dict]:
    cases, cur = [], {}
    with open(os.path.join(GOLDEN, "thresholds_rule.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("#"):
                continue
            if not line:
                if cur:
                    cases.append(cur)
                cur = {}
                continue
            k, v = _parse_line(line)
            cur[k] = v
    if cur:
        cases.append(cur)
    out = []
    for c in cases:
        out.append(dict(name=c["name"][0],
                        sum=np.array([int(x) for x in c["sum"]], np.int64),
                        count=np.array([int(x) for x in c["count"]], np.int64),
                        thresholds=[int(x) for x in c.get("thresholds", [])],
                        t0=int(c["t0"][0])))
    return out


def pin_golden(lib=None, name: str | None = None):
    for fname in ([name] if name else curve_fixture_names()):
        fx = load_curve_fixture(fname)
        s, k, c = oracle.curve(fx["image"], fx["M"], fx["nbhd"], lib=lib)
        assert np.array_equal(s, fx["sum"]), (fname, "sum", s, fx["sum"])
        assert np.array_equal(k, fx["count"]), (fname, "count", k, fx["count"])
        for t, q in enumerate(fx["C"]):
            assert c[t] == float(q), (fname, "C", t, c[t], q)
        thr, t0, _, _ = oracle.thresholds(s, k, lib=lib)
        assert list(thr) == fx["thresholds"], (fname, "thresholds", thr, fx["thresholds"])
        assert t0 == fx["t0"], (fname, "t0", t0, fx["t0"])


def pin_threshold_rule(lib=None):
    for case in load_threshold_cases():
        thr, t0, st, n = oracle.thresholds(case["sum"], case["count"], lib=lib)
        assert list(thr) == case["thresholds"], (case["name"], thr)
        assert t0 == case["t0"], (case["name"], t0)
        assert st == oracle.OK and n == len(case["thresholds"])


# ----------------------------------------------------------------------------------------------
# closed forms, special cases, symmetries, bounds

HALF4 = [(0, 1), (1, 0)]
HALF8 = HALF4 + [(1, 1), (1, -1)]


def pair_gaps(img: np.ndarray, nbhd: int) -> np.ndarray:
    """|f(p) - f(q)| for every unordered neighbour pair, enumerated by array slicing."""
    f = np.asarray(img, dtype=np.int64)
    H, W = f.shape
    out = []
    for dy, dx in (HALF4 if nbhd == 4 else HALF8):
        ys0, ys1 = slice(0, H - dy), slice(dy, H)
        if dx >= 0:
            xs0, xs1 = slice(0, W - dx), slice(dx, W)
        else:
            xs0, xs1 = slice(-dx, W), slice(0, W + dx)
        out.append(np.abs(f[ys0, xs0] - f[ys1, xs1]).ravel())
    return np.concatenate(out) if out else np.zeros(0, np.int64)


def pin_closed_form_totals(lib=None, seeds=range(6)):
    for seed in seeds:
        rng = np.random.default_rng(1000 + seed)
        for nbhd in (4, 8):
            H, W = int(rng.integers(1, 20)), int(rng.integers(1, 20))
            M = int(rng.choice([2, 3, 7, 16, 64, 256]))
            img = rng.integers(0, M, size=(H, W))
            s, k, _ = oracle.curve(img, M, nbhd, lib=lib)
            d = pair_gaps(img, nbhd)
            assert int(k.sum()) == int(d.sum()), ("sum count", seed, nbhd)
            assert int(s.sum()) == int((d * d // 4).sum()), ("sum sum", seed, nbhd)


def pin_special_cases(lib=None):
    rng = np.random.default_rng(7)
    # constant image: every pair has gap 0, so B(t) is empty for every t
    for nbhd in (4, 8):
        img = np.full((5, 7), 3)
        s, k, c = oracle.curve(img, 8, nbhd, lib=lib)
        assert not s.any() and not k.any() and not c.any()
        thr, t0, _, _ = oracle.thresholds(s, k, lib=lib)
        assert len(thr) == 0 and t0 == -1
    # two-level image {a < b}: count(t) = P_ab and sum(t) = P_ab * min(b - t, t - a) on [a, b-1]
    for a, b, M in [(2, 9, 12), (0, 1, 2), (5, 6, 10), (3, 10, 16), (1, 7, 8), (0, 255, 256)]:
        for nbhd in (4, 8):
            img = np.where(rng.integers(0, 2, size=(6, 9)) == 1, b, a)
            P = int((pair_gaps(img, nbhd) > 0).sum())
            s, k, c = oracle.curve(img, M, nbhd, lib=lib)
            for t in range(M):
                inside = a <= t < b
                assert k[t] == (P if inside else 0), (a, b, t)
                assert s[t] == (P * min(b - t, t - a) if inside else 0), (a, b, t)
            thr, t0, _, _ = oracle.thresholds(s, k, lib=lib)
            if P and b - a >= 2:
                assert list(thr) == [(a + b) // 2] and t0 == (a + b) // 2, (a, b, thr, t0)
            else:
                assert len(thr) == 0 and t0 == -1
    # unit ramp along rows: every pair has gap 0 or 1, and a gap-1 pair has contrast 0
    img = np.tile(np.arange(12), (4, 1))
    s, k, c = oracle.curve(img, 16, 4, lib=lib)
    assert not s.any() and not c.any()
    assert list(k[:11]) == [4] * 11 and not k[11:].any()


def pin_symmetries(lib=None, seeds=range(4)):
    for seed in seeds:
        rng = np.random.default_rng(2000 + seed)
        H, W = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        M = int(rng.choice([5, 16, 33]))
        img = rng.integers(0, M, size=(H, W))
        for nbhd in (4, 8):
            s, k, _ = oracle.curve(img, M, nbhd, lib=lib)
            for g in (img.T, img[::-1], img[:, ::-1], img[::-1, ::-1]):
                s2, k2, _ = oracle.curve(g, M, nbhd, lib=lib)
                assert np.array_equal(s, s2) and np.array_equal(k, k2), ("geometric", seed, nbhd)
            # inversion g = M-1-f: sum_g(t) = sum_f(M-1-t), count_g(t) = count_f(M-2-t)
            si, ki, _ = oracle.curve(M - 1 - img, M, nbhd, lib=lib)
            assert np.array_equal(si, s[::-1]), ("inversion sum", seed, nbhd)
            kf = np.concatenate([k[::-1][1:], [0]])  # count_f(M-2-t), with count_f(-1) = 0
            assert np.array_equal(ki, kf), ("inversion count", seed, nbhd)
            # shift g = f + c without clipping: both curves move right by c
            cshift = 3
            ss, ks, _ = oracle.curve(img + cshift, M + cshift, nbhd, lib=lib)
            assert np.array_equal(ss[cshift:], s) and not ss[:cshift].any(), ("shift", seed)
            assert np.array_equal(ks[cshift:], k) and not ks[:cshift].any(), ("shift", seed)


def pin_bounds(lib=None, seeds=range(4)):
    for seed in seeds:
        rng = np.random.default_rng(3000 + seed)
        M = int(rng.choice([4, 16, 256]))
        img = rng.integers(0, M, size=(int(rng.integers(1, 12)), int(rng.integers(1, 12))))
        for nbhd in (4, 8):
            s, k, c = oracle.curve(img, M, nbhd, lib=lib)
            t = np.arange(M)
            assert k[M - 1] == 0 and s[M - 1] == 0
            assert np.all(c >= 0) and np.all(c <= np.minimum(t, M - 1 - t))
            assert np.all(c[k == 0] == 0)


# ----------------------------------------------------------------------------------------------
# two other routes to the same integers

def pin_alg1(lib=None, seeds=range(8)):
    """Eq (9): Algorithm 1 over the half neighbourhood equals the full ordered-pair definition."""
    for seed in seeds:
        rng = np.random.default_rng(4000 + seed)
        M = int(rng.choice([2, 5, 16, 64, 256]))
        img = rng.integers(0, M, size=(int(rng.integers(1, 16)), int(rng.integers(1, 16))))
        for nbhd in (4, 8):
            s, k, _ = oracle.curve(img, M, nbhd, lib=lib)
            s1, k1 = oracle.alg1(img, M, nbhd, lib=lib)
            assert np.array_equal(s, s1) and np.array_equal(k, k1), ("alg1", seed, nbhd)


def direct_by_dilation(img: np.ndarray, M: int, nbhd: int):
    """The direct route of Sec. 3.1 in plain Python: for each t, the pixels x0 of the boundary are
    (C_1 dilated by the neighbourhood) minus C_1 (eqs (5)-(6)); each such x0 is paired with its
    neighbours in C_1 and the contrasts of eq (2) are added up. Exact fractions for C."""
    H, W = img.shape
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    if nbhd == 8:
        offs += [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    sums, counts = [], []
    for t in range(M):
        c1 = {(y, x) for y in range(H) for x in range(W) if img[y, x] > t}
        dil = {(y + dy, x + dx) for (y, x) in c1 for (dy, dx) in offs
               if 0 <= y + dy < H and 0 <= x + dx < W}
        border = dil - c1
        S = K = 0
        for (y, x) in border:
            for (dy, dx) in offs:
                q = (y + dy, x + dx)
                if q in c1:
                    S += min(int(img[q]) - t, t - int(img[y, x]))
                    K += 1
        sums.append(S)
        counts.append(K)
    return np.array(sums, np.int64), np.array(counts, np.int64)


def pin_direct_dilation(lib=None, seeds=range(10)):
    for seed in seeds:
        rng = np.random.default_rng(5000 + seed)
        M = int(rng.choice([2, 3, 5, 8]))
        img = rng.integers(0, M, size=(int(rng.integers(1, 6)), int(rng.integers(1, 6))))
        for nbhd in (4, 8):
            s, k, _ = oracle.curve(img, M, nbhd, lib=lib)
            sd, kd = direct_by_dilation(img, M, nbhd)
            assert np.array_equal(s, sd) and np.array_equal(k, kd), ("dilation", seed, nbhd)


# ----------------------------------------------------------------------------------------------
# other neighbourhoods: a symmetric structuring element A with half A*, and the hexagonal grid

N4_FULL = [(-1, 0), (1, 0), (0, -1), (0, 1)]
N8_FULL = N4_FULL + [(-1, -1), (-1, 1), (1, -1), (1, 1)]


def hex_neighbours(y: int) -> list[tuple[int, int]]:
    """The hexagonal grid's neighbour offsets in row y, odd rows shifted right by half a pixel:
    two in the row, and the two pixels of each adjacent row that touch this one (for an even row
    the one below-left and the one below, as the odd row below sits half a pixel to the right)."""
    if y % 2 == 0:
        return [(0, -1), (0, 1), (-1, -1), (-1, 0), (1, -1), (1, 0)]
    return [(0, -1), (0, 1), (-1, 0), (-1, 1), (1, 0), (1, 1)]


def nbhd_pairs(img: np.ndarray, offs_of_row) -> list[tuple[int, int]]:
    """Every unordered neighbour pair {p, q} once, as (f(p), f(q)), for a neighbourhood given by its
    full offsets per row; the relation is symmetric, so each pair is seen from both ends and kept
    from the end that comes first in raster order."""
    H, W = img.shape
    out = []
    for y in range(H):
        for x in range(W):
            for dy, dx in offs_of_row(y):
                y1, x1 = y + dy, x + dx
                if 0 <= y1 < H and 0 <= x1 < W and (y1, x1) > (y, x):
                    out.append((int(img[y, x]), int(img[y1, x1])))
    return out


def load_nbhd_fixture(name: str) -> dict:
    d: dict = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = _parse_line(line)
            d[k] = v
    H, W = int(d["H"][0]), int(d["W"][0])
    o = [int(x) for x in d.get("offsets", [])]
    return dict(image=np.array([int(x) for x in d["image"]], dtype=np.int64).reshape(H, W),
                M=int(d["M"][0]), hex=int(d["hex"][0]) == 1, offsets=list(zip(o[0::2], o[1::2])),
                sum=np.array([int(x) for x in d["sum"]], np.int64),
                count=np.array([int(x) for x in d["count"]], np.int64),
                C=[Fraction(x) for x in d["C"]], thresholds=[int(x) for x in d.get("thresholds", [])],
                t0=int(d["t0"][0]))


def nbhd_fixture_names() -> list[str]:
    return sorted(f for f in os.listdir(GOLDEN) if f.startswith("n") and f.endswith(".txt"))


def pin_nbhd_golden(lib=None):
    for fname in nbhd_fixture_names():
        fx = load_nbhd_fixture(fname)
        s, k, c = oracle.curve_nbhd(fx["image"], fx["M"], offsets=fx["offsets"], hex=fx["hex"], lib=lib)
        assert np.array_equal(s, fx["sum"]) and np.array_equal(k, fx["count"]), (fname, s, k)
        assert [float(q) for q in fx["C"]] == list(c), (fname, "C", c)
        thr, t0, _, _ = oracle.thresholds(s, k, lib=lib)
        assert list(thr) == fx["thresholds"] and t0 == fx["t0"], (fname, thr, t0)
        half = None if fx["hex"] else oracle.half_of(fx["offsets"])
        s1, k1 = oracle.alg1_nbhd(fx["image"], fx["M"], half=half, hex=fx["hex"], lib=lib)
        assert np.array_equal(s1, fx["sum"]) and np.array_equal(k1, fx["count"]), (fname, "alg1")


def random_half(rng, n_max: int = 6, r: int = 3) -> list[tuple[int, int]]:
    """A random half set: distinct offsets with dy > 0, or dy == 0 and dx > 0, within radius r."""
    cand = [(dy, dx) for dy in range(0, r + 1) for dx in range(-r, r + 1) if dy > 0 or dx > 0]
    idx = rng.choice(len(cand), size=int(rng.integers(1, n_max + 1)), replace=False)
    return [cand[i] for i in sorted(idx)]


def pin_nbhd_alg1(lib=None, seeds=range(8)):
    """Eq (9) for a symmetric A and for the hexagonal grid: the full ordered-pair definition equals
    Algorithm 1 over the half."""
    for seed in seeds:
        rng = np.random.default_rng(6000 + seed)
        M = int(rng.choice([2, 5, 16, 64, 256]))
        img = rng.integers(0, M, size=(int(rng.integers(1, 14)), int(rng.integers(1, 14))))
        half = random_half(rng)
        s, k, _ = oracle.curve_nbhd(img, M, offsets=oracle.full_of(half), lib=lib)
        s1, k1 = oracle.alg1_nbhd(img, M, half=half, lib=lib)
        assert np.array_equal(s, s1) and np.array_equal(k, k1), ("alg1 offsets", seed, half)
        s, k, _ = oracle.curve_nbhd(img, M, hex=True, lib=lib)
        s1, k1 = oracle.alg1_nbhd(img, M, hex=True, lib=lib)
        assert np.array_equal(s, s1) and np.array_equal(k, k1), ("alg1 hex", seed)


def pin_nbhd_closed_forms(lib=None, seeds=range(6)):
    """Over thresholds, sum_t #B(t) = sum of the gaps and sum_t sum(t) = sum of floor(d^2/4), with
    the pairs listed independently (nbhd_pairs); and an isolated pixel of an otherwise constant
    image has as many pairs as neighbours (6 inside the hexagonal grid)."""
    for seed in seeds:
        rng = np.random.default_rng(6100 + seed)
        M = int(rng.choice([3, 16, 256]))
        img = rng.integers(0, M, size=(int(rng.integers(1, 12)), int(rng.integers(1, 12))))
        half = random_half(rng)
        full = oracle.full_of(half)
        for offs_of_row, kw in ((lambda y: full, dict(offsets=full)), (hex_neighbours, dict(hex=True))):
            d = np.array([abs(a - b) for a, b in nbhd_pairs(img, offs_of_row)], np.int64)
            s, k, _ = oracle.curve_nbhd(img, M, lib=lib, **kw)
            assert int(k.sum()) == int(d.sum()), ("count total", seed, kw)
            assert int(s.sum()) == int((d * d // 4).sum()), ("sum total", seed, kw)
    for y, x in [(2, 3), (3, 3), (0, 3), (3, 0), (5, 6)]:
        img = np.zeros((6, 7), np.int64)
        img[y, x] = 9
        _, k, _ = oracle.curve_nbhd(img, 10, hex=True, lib=lib)
        deg = sum(1 for dy, dx in hex_neighbours(y) if 0 <= y + dy < 6 and 0 <= x + dx < 7)
        assert list(k[:9]) == [deg] * 9 and not k[9:].any(), ("isolated pixel", y, x, deg)
        if 0 < y < 5 and 0 < x < 6:
            assert deg == 6


def pin_nbhd_reductions(lib=None, seeds=range(4)):
    """The offset sets of N4 and N8 give the 4- and 8-neighbourhood curves; the hexagonal grid on a
    single row or a single column has only N4's pairs."""
    for seed in seeds:
        rng = np.random.default_rng(6200 + seed)
        M = int(rng.choice([4, 32, 256]))
        img = rng.integers(0, M, size=(int(rng.integers(1, 10)), int(rng.integers(1, 10))))
        for full, nbhd in ((N4_FULL, 4), (N8_FULL, 8)):
            s, k, c = oracle.curve_nbhd(img, M, offsets=full, lib=lib)
            s0, k0, c0 = oracle.curve(img, M, nbhd, lib=lib)
            assert np.array_equal(s, s0) and np.array_equal(k, k0) and np.array_equal(c, c0), (seed, nbhd)
        for line in (img[:1], img[:, :1]):
            s, k, _ = oracle.curve_nbhd(line, M, hex=True, lib=lib)
            s0, k0, _ = oracle.curve(line, M, 4, lib=lib)
            assert np.array_equal(s, s0) and np.array_equal(k, k0), ("hex line", seed, line.shape)


def direct_by_dilation_rows(img: np.ndarray, M: int, offs_of_row):
    """The direct route of Sec. 3.1 for a neighbourhood given per row: boundary pixels x0 are the
    neighbours of C_1^t outside C_1^t, each paired with its neighbours in C_1^t."""
    H, W = img.shape
    sums, counts = [], []
    for t in range(M):
        c1 = {(y, x) for y in range(H) for x in range(W) if img[y, x] > t}
        border = {(y + dy, x + dx) for (y, x) in c1 for (dy, dx) in offs_of_row(y)
                  if 0 <= y + dy < H and 0 <= x + dx < W} - c1
        S = K = 0
        for (y, x) in border:
            for (dy, dx) in offs_of_row(y):
                q = (y + dy, x + dx)
                if q in c1:
                    S += min(int(img[q]) - t, t - int(img[y, x]))
                    K += 1
        sums.append(S)
        counts.append(K)
    return np.array(sums, np.int64), np.array(counts, np.int64)


def pin_nbhd_direct(lib=None, seeds=range(6)):
    for seed in seeds:
        rng = np.random.default_rng(6300 + seed)
        M = int(rng.choice([2, 3, 5, 8]))
        img = rng.integers(0, M, size=(int(rng.integers(1, 6)), int(rng.integers(1, 6))))
        full = oracle.full_of(random_half(rng, n_max=4, r=2))
        for offs_of_row, kw in ((lambda y: full, dict(offsets=full)), (hex_neighbours, dict(hex=True))):
            s, k, _ = oracle.curve_nbhd(img, M, lib=lib, **kw)
            sd, kd = direct_by_dilation_rows(img, M, offs_of_row)
            assert np.array_equal(s, sd) and np.array_equal(k, kd), ("direct", seed, kw)


ALL_PINS = [pin_golden, pin_threshold_rule, pin_closed_form_totals, pin_special_cases,
            pin_symmetries, pin_bounds, pin_alg1, pin_direct_dilation, pin_nbhd_golden, pin_nbhd_alg1,
            pin_nbhd_closed_forms, pin_nbhd_reductions, pin_nbhd_direct]


# ----------------------------------------------------------------------------------------------
# the 3x3 binomial pre-filter (Python oracle)

def load_filter_cases() -> list[dict]:
    cases, cur = [], {}
    with open(os.path.join(GOLDEN, "f1_binomial3.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("#"):
                continue
            if not line:
                if cur:
                    cases.append(cur)
                cur = {}
                continue
            k, v = _parse_line(line)
            cur[k] = v
    if cur:
        cases.append(cur)
    out = []
    for c in cases:
        H, W = int(c["H"][0]), int(c["W"][0])
        out.append(dict(name=c["case"][0], image=np.array([int(x) for x in c["image"]], np.uint8).reshape(H, W),
                        out=np.array([int(x) for x in c["out"]], np.uint8).reshape(H, W)))
    return out


def pin_binomial3(filt=None, seeds=range(6)):
    filt = filt or oracle.binomial3
    for case in load_filter_cases():
        assert np.array_equal(filt(case["image"]), case["out"]), case["name"]
    # constant images are unchanged (weights add up to 16)
    for v in (0, 1, 7, 255):
        assert np.array_equal(filt(np.full((4, 5), v, np.uint8)), np.full((4, 5), v, np.uint8))
    # impulse response: 16 at an interior pixel of zeros gives the kernel itself
    imp = np.zeros((5, 5), np.uint16)
    imp[2, 2] = 16
    want = np.zeros((5, 5), np.uint16)
    want[1:4, 1:4] = [[1, 2, 1], [2, 4, 2], [1, 2, 1]]
    assert np.array_equal(filt(imp), want)
    for seed in seeds:
        rng = np.random.default_rng(6400 + seed)
        H, W = int(rng.integers(1, 12)), int(rng.integers(1, 12))
        img = rng.integers(0, 4096, size=(H, W)).astype(np.uint16)
        g = filt(img)
        # the separable route: [1 2 1] down the columns then along the rows, rounded once
        f = np.pad(img.astype(np.int64), 1, mode="edge")
        v = f[:-2] + 2 * f[1:-1] + f[2:]
        hsum = v[:, :-2] + 2 * v[:, 1:-1] + v[:, 2:]
        assert np.array_equal(g.astype(np.int64), (hsum + 8) // 16), ("separable", seed)
        assert np.array_equal(filt(img.T), g.T), ("transpose", seed)
        assert g.min() >= img.min() and g.max() <= img.max(), ("range", seed)
        assert g.dtype == img.dtype and g.shape == img.shape


# ------------------------------------------------------------------------------------------------
# segmentation by the thresholds (Sec. 2.1: the lower set of t is {f <= t})

def pin_segment():
    """Hand cases, the library routine it reduces to, and invariants of the class labels."""
    import oracle
    # W1: f = [0, 4, 1] with threshold {2}: 0 and 1 lie in {f <= 2}, 4 does not
    assert oracle.segment(np.array([[0, 4, 1]]), [2]).tolist() == [[0, 1, 0]]
    # W2 with its threshold {3}
    w2 = np.array([[0, 0, 5], [2, 7, 5]])
    assert oracle.segment(w2, [3]).tolist() == [[0, 0, 1], [0, 1, 1]]
    # a value equal to a threshold stays below it; two thresholds give three classes
    assert oracle.segment(np.array([[2, 3, 4, 6, 7]]), [3, 6]).tolist() == [[0, 0, 1, 1, 2]]
    # no thresholds: one class
    assert oracle.segment(np.array([[0, 9, 255]]), []).tolist() == [[0, 0, 0]]
    rng = np.random.default_rng(5)
    for _ in range(20):
        M = int(rng.integers(2, 300))
        k = int(rng.integers(0, min(M, 12)))
        thr = np.sort(rng.choice(M, size=k, replace=False))
        img = rng.integers(0, M, size=(int(rng.integers(1, 40)), int(rng.integers(1, 40))))
        lab = oracle.segment(img, thr)
        # the count of thresholds below f is numpy's left insertion point
        assert np.array_equal(lab, np.searchsorted(thr, img, side="left"))
        # labels grow with the value and stay in [0, k]
        order = np.argsort(img, axis=None, kind="stable")
        assert np.all(np.diff(lab.reshape(-1)[order]) >= 0)
        assert lab.min() >= 0 and lab.max() <= k
        # class i holds exactly the values in (t_i, t_{i+1}]
        for i in range(k + 1):
            lo = -1 if i == 0 else thr[i - 1]
            hi = M if i == k else thr[i]
            assert np.array_equal(lab == i, (img > lo) & (img <= hi))


def pin_class_stats():
    """Class counts, sums and means by hand, by brute force over pixels and by invariants; the mean
    image; the most significant thresholds by hand and against a float sort where C values are far
    apart."""
    import oracle
    # W1 = [0, 4, 1], threshold {2}: class 0 holds 0 and 1, class 1 holds 4
    c, s, m = oracle.class_stats(np.array([[0, 4, 1]]), [2], 5)
    assert c.tolist() == [2, 1] and s.tolist() == [1, 4] and m.tolist() == [0.5, 4.0]
    # the class means 0.5 and 4.0 round to 0 (ties to even) and 4
    assert oracle.mean_image(np.array([[0, 4, 1]], np.uint8), [2], 5).tolist() == [[0, 4, 0]]
    # an empty middle class has mean 0; a value >= M counts in the top class as M
    c, s, m = oracle.class_stats(np.array([[1, 9, 300]]), [3, 5], 256)
    assert c.tolist() == [1, 0, 2] and s.tolist() == [1, 0, 265] and m.tolist() == [1.0, 0.0, 132.5]
    # no thresholds: one class, the image mean
    c, s, m = oracle.class_stats(np.array([[2, 3], [4, 7]]), [], 8)
    assert c.tolist() == [4] and s.tolist() == [16] and m.tolist() == [4.0]
    rng = np.random.default_rng(11)
    for _ in range(20):
        M = int(rng.integers(2, 300))
        k = int(rng.integers(0, min(M, 12)))
        thr = np.sort(rng.choice(M, size=k, replace=False))
        img = rng.integers(0, M, size=(int(rng.integers(1, 30)), int(rng.integers(1, 30))))
        c, s, m = oracle.class_stats(img, thr, M)
        # brute force: walk the pixels, find each one's class by scanning the thresholds
        bc = [0] * (k + 1)
        bs = [0] * (k + 1)
        for v in img.reshape(-1).tolist():
            j = 0
            while j < k and thr[j] < v:
                j += 1
            bc[j] += 1
            bs[j] += v
        assert c.tolist() == bc and s.tolist() == bs
        # invariants: every pixel counted once, the class means weighted by counts give the image sum,
        # and a non-empty class's mean lies inside its interval (t_{j-1}, t_j]
        assert c.sum() == img.size and s.sum() == img.sum()
        for j in range(k + 1):
            if c[j]:
                lo = -1 if j == 0 else thr[j - 1]
                hi = M - 1 if j == k else thr[j]
                assert lo < m[j] <= hi
                assert abs(m[j] * c[j] - s[j]) <= 1e-9 * max(1, s[j])
            else:
                assert m[j] == 0.0
        mi = oracle.mean_image(img.astype(np.uint16), thr, M)
        lab = oracle.segment(img, thr)
        assert np.array_equal(mi, np.rint(m)[lab].astype(np.uint16))

    # most significant thresholds: C = [0, 3/2, 1, 3/2, 2, 0]; the maxima 1 and 4 (and 3) in order of C
    s_ = np.array([0, 3, 2, 3, 4, 0])
    k_ = np.array([1, 2, 2, 2, 2, 0])
    assert oracle.top_thresholds(s_, k_, [1, 3, 4], 2) == [4, 1]   # 2 first, then the tie 1 < 3
    assert oracle.top_thresholds(s_, k_, [1, 3, 4], 5) == [4, 1, 3]
    assert oracle.top_thresholds(s_, k_, [1, 3, 4], 0) == []
    assert oracle.top_thresholds(s_, k_, [5, 1], 2) == [1, 5]      # count 0 reads as C = 0
    # exact order where the doubles tie: 2^53 and 2^53 + 1 (over 1) are one double, so a float
    # comparison would fall back to the smaller t
    big = np.array([2 ** 53, 2 ** 53 + 1], dtype=np.int64)
    assert oracle.top_thresholds(big, np.array([1, 1]), [0, 1], 1) == [1]
    rng = np.random.default_rng(12)
    for _ in range(20):
        n = int(rng.integers(1, 40))
        cnt = rng.integers(2, 1000, size=n)
        C = rng.permutation(n).astype(np.float64) + 0.5     # distinct, at least 1 apart
        sm = np.rint(C * cnt).astype(np.int64)               # sum / count within 1/4 of C
        thr = sorted(rng.choice(n, size=int(rng.integers(0, n + 1)), replace=False).tolist())
        kk = int(rng.integers(0, n + 2))
        want = sorted(thr, key=lambda t: -C[t])[:kk]
        assert oracle.top_thresholds(sm, cnt, thr, kk) == want
