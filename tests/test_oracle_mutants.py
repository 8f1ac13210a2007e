"""Plant plausible mistakes in a copy of the oracle's C source and check that the pins catch each.

The committed oracle is never modified: every mutant is a textual edit of a temporary copy, built
with the same compiler flags, and run on the CPU only.
"""
import os

import pytest

import _pins
import oracle

MUTANTS = {
    # eq (1): x0 in C_0^t means f(x0) <= t, x1 in C_1^t means f(x1) > t
    "c0_strict": ("if (f0 > t) /* x0 must lie in C_0^t */", "if (f0 >= t) /* x0 must lie in C_0^t */"),
    "c1_nonstrict": ("if (f1 <= t) /* x1 must lie in C_1^t */", "if (f1 < t) /* x1 must lie in C_1^t */"),
    # eq (2): the minimum of the two steps, with the right signs
    "max_not_min": ("S += up < down ? up : down;", "S += up < down ? down : up;"),
    "step_off_by_one": ("const int64_t up = f1 - t, down = t - f0; /* eq (2) */",
                        "const int64_t up = f1 - t, down = t - f0 + 1; /* eq (2) */"),
    "dropped_count": ("K += 1;\n                }", "K += 0;\n                }"),
    # eq (3): numerator and denominator
    "transposed_division": ("C[k] = K ? (double)S / (double)K : 0.0;", "C[k] = S ? (double)K / (double)S : 0.0;"),
    # the neighbourhood: a wrong offset index
    "wrong_offset": ("static const int NB_DY[8] = {-1, 1, 0, 0, -1, -1, 1, 1};",
                     "static const int NB_DY[8] = {-1, -1, 0, 0, -1, -1, 1, 1};"),
    # Algorithm 1's threshold range [lo, hi-1]
    "alg1_range": ("for (int64_t t = lo; t < hi; t++) {", "for (int64_t t = lo; t <= hi && t < M; t++) {"),
    # threshold rule: report the run's first threshold; ties of eq (4) go to the smallest t
    "report_run_end": ("thr[found] = a;", "thr[found] = b;"),
    "t0_last_tie": ("if (cmp_curve(sum[t], count[t], sum[best], count[best]) > 0)",
                    "if (cmp_curve(sum[t], count[t], sum[best], count[best]) >= 0)"),
    "float_compare": ("const __int128 l = nu * dv, r = nv * du;",
                      "const __int128 l = (__int128)((double)nu / (double)du * 1e18), r = (__int128)((double)nv / (double)dv * 1e18);"),
    # other neighbourhoods: the hexagonal grid's row parity, its half, and a generic offset's sign
    "hex_parity_swapped": ("const int odd = (int)(y & 1);", "const int odd = (int)((y + 1) & 1);"),
    "hex_half_wrong_diagonal": ("static const int HEY[3] = {0, 1, 1}, HEX_[3] = {1, -1, 0};",
                                "static const int HEY[3] = {0, 1, 1}, HEX_[3] = {1, 1, 0};"),
    "nbhd_offset_sign": ("const int64_t y1 = y + ody[a], x1 = x + odx[a];",
                         "const int64_t y1 = y + ody[a], x1 = x - odx[a];"),
    "nbhd_max_not_min": ("S += rise < fall ? rise : fall;", "S += rise < fall ? fall : rise;"),
    "nbhd_alg1_range": ("for (int64_t t = lo; t < hi; ++t) { /* lo <= t < hi */",
                        "for (int64_t t = lo + 1; t < hi; ++t) { /* lo <= t < hi */"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = oracle.build(str(path), str(tmp_path / "libmutant.so"))
    lib = oracle.load_library(so)
    caught = []
    for pin in _pins.ALL_PINS:
        try:
            pin(lib)
        except (AssertionError, oracle.OracleError) as e:
            caught.append((pin.__name__, str(e)[:80]))
    assert caught, f"mutant {name} passed every pin"


# Mistakes planted in the oracle's Python functions (segmentation and its consumers): each is a
# textual edit of the function's source, compiled into a copy of the module's namespace and swapped
# in for the duration of the test only.
PY_MUTANTS = {
    # Sec. 2.1 / eq (1): a value equal to a threshold lies in the threshold's lower set
    "segment_nonstrict": ("segment", "(blk[..., None] > t[None, None, :])", "(blk[..., None] >= t[None, None, :])"),
    # class mean: sum over count
    "class_mean_transposed": ("class_stats", "mean[j] = np.float64(total[j]) / np.float64(count[j])",
                              "mean[j] = np.float64(count[j]) / np.float64(total[j])"),
    # values >= M count at the value M
    "class_clamp_below_M": ("class_stats", "f = np.minimum(np.asarray(img).astype(np.int64), M)",
                            "f = np.minimum(np.asarray(img).astype(np.int64), M - 1)"),
    # rounding of the class means: ties to even
    "mean_round_half_up": ("mean_image", "return np.rint(mean)[lab].astype(img.dtype)",
                           "return np.floor(mean + 0.5)[lab].astype(img.dtype)"),
    # most significant thresholds: exact order, equal C in ascending t
    "top_float_order": ("top_thresholds", "return (-(Fraction(int(sum_[t]), c) if c else Fraction(0)), int(t))",
                        "return (-(int(sum_[t]) / c if c else 0.0), int(t))"),
    "top_tie_larger_t": ("top_thresholds", "return (-(Fraction(int(sum_[t]), c) if c else Fraction(0)), int(t))",
                         "return (-(Fraction(int(sum_[t]), c) if c else Fraction(0)), -int(t))"),
    # the binomial pre-filter: round half up, replicated borders, the weights
    "binomial_floor": ("binomial3", "return ((acc + 8) // 16).astype(a.dtype)", "return (acc // 16).astype(a.dtype)"),
    "binomial_wrap": ("binomial3", "ys = np.clip(np.arange(H) + i, 0, H - 1)", "ys = (np.arange(H) + i) % H"),
    "binomial_box": ("binomial3", "acc += BINOMIAL3[i + 1][j + 1] * f[ys][:, xs]", "acc += 16 * f[ys][:, xs] // 9"),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_python_mutant_is_caught(name, monkeypatch):
    import inspect
    import textwrap

    fn, old, new = PY_MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(getattr(oracle, fn)))
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), ns)
    monkeypatch.setattr(oracle, fn, ns[fn])
    caught = []
    for pin in (_pins.pin_segment, _pins.pin_class_stats, _pins.pin_binomial3):
        try:
            pin()
        except AssertionError as e:
            caught.append((pin.__name__, str(e)[:80]))
    assert caught, f"mutant {name} passed every pin"


@pytest.mark.parametrize("fn", sorted({v[0] for v in PY_MUTANTS.values()}))
def test_python_unmutated_copy_passes(fn, monkeypatch):
    """Control: the same recompilation without an edit passes every pin, so a caught mutant is caught
    for its edit."""
    import inspect
    import textwrap

    ns = dict(vars(oracle))
    exec(compile(textwrap.dedent(inspect.getsource(getattr(oracle, fn))), f"<copy {fn}>", "exec"), ns)
    monkeypatch.setattr(oracle, fn, ns[fn])
    _pins.pin_segment()
    _pins.pin_class_stats()
    _pins.pin_binomial3()
