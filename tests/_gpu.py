"""Helpers for the GPU parity tests: compare library results with the CPU oracle.

The bar: sum and count bit-exact (integer work), thresholds and t0 identical (decided by exact
rational comparisons on both sides), C within 1e-12 relative (both sides divide the same two exact
integers with one IEEE binary64 division, so 0 ulp is expected and checked separately)."""
from __future__ import annotations

import sys

import numpy as np

import oracle

C_RTOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def reference(img, M, nbhd, exact_all=True):
    """Oracle result: the brute force of eqs (1)-(3) when feasible, else Algorithm 1 (both pinned)."""
    if exact_all:
        s, k, _ = oracle.curve(img, M, nbhd)
    else:
        s, k = oracle.alg1(img, M, nbhd)
    c = np.where(k > 0, s.astype(np.float64) / np.where(k > 0, k, 1).astype(np.float64), 0.0)
    thr, t0, _, n = oracle.thresholds(s, k)
    return dict(sum=s, count=k, C=c, thr=thr, t0=t0, n=n)


def assert_same(got_sum, got_count, got_C, got_thr, got_t0, got_n, ref, cap=None, what=""):
    got_sum = np.asarray(got_sum)
    got_count = np.asarray(got_count)
    got_C = np.asarray(got_C)
    assert np.array_equal(got_sum, ref["sum"]), f"{what}: sum differs at {np.nonzero(got_sum != ref['sum'])[0][:10]}"
    assert np.array_equal(got_count, ref["count"]), f"{what}: count differs at {np.nonzero(got_count != ref['count'])[0][:10]}"
    np.testing.assert_allclose(got_C, ref["C"], rtol=C_RTOL, atol=0, err_msg=what)
    assert np.array_equal(got_C, ref["C"]), f"{what}: C not bit-identical (expected 0 ulp)"
    cap = len(ref["thr"]) if cap is None else cap
    assert got_n == ref["n"], f"{what}: n_thresholds {got_n} != {ref['n']}"
    assert list(np.asarray(got_thr)[: min(cap, got_n)]) == list(ref["thr"][:cap]), f"{what}: thresholds differ"
    assert got_t0 == ref["t0"], f"{what}: t0 {got_t0} != {ref['t0']}"


def assert_result(res, ref, cap=None, what=""):
    assert_same(res.sum, res.count, res.C, res.thresholds, res.t0, res.n_thresholds, ref, cap, what)


def to_device(img):
    import torch
    a = np.ascontiguousarray(img)
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16)).cuda().view(torch.uint16)
    return torch.from_numpy(a).cuda()
