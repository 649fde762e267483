"""Pins of the oracle's sparsity pattern, prefix sum and state comparison.

* nnz from the brute-force pattern equals a class-pair count that never forms
  a state pair (Sec. 2.1 rule popcount <= 4 applied per species);
* every operator-generated entry has popcount(xor) in {0, 2, 4} (Sec. 2.1);
* count_difference (Listing 1 as a description) equals popcount of the xor;
* the serial counts-to-offsets recurrence (Sec. 2.2) equals the running
  totals of the standard library, including totals beyond 2^32.
"""
import itertools

import numpy as np
import pytest

import cigen
import oracle as O


@pytest.mark.parametrize("name", ["sp1_n2_N4", "ab_n3_3p3_cut4"])
def test_nnz_matches_class_count(name):
    w = cigen.WORKLOADS[name]
    b = O.Basis(w.spec)
    ptr, _ = O.pattern_rows(b)
    full, half = O.nnz_class_count(w.spec)
    assert int(ptr[-1]) == half
    assert half == (full + b.D) // 2
    want = {"sp1_n2_N4": 63213, "ab_n3_3p3_cut4": 3552476}[name]
    assert half == want


def test_random_small_specs_nnz():
    rng = np.random.default_rng(11)
    for _ in range(8):
        spec = cigen.random_spec_small(rng)
        try:
            b = O.Basis(spec)
        except ValueError:
            continue
        if b.D == 0:
            continue
        ptr, _ = O.pattern_rows(b)
        assert int(ptr[-1]) == O.nnz_class_count(spec)[1], spec


def test_operator_entries_are_inside_the_pattern_and_even():
    w = cigen.WORKLOADS["sp1_n2_N4"]
    b = O.Basis(w.spec)
    H = O.dense_H(b, O.Interaction(b, cigen.make_tables(w.spec, w.seed)))
    g = b.glob
    for i in range(0, b.D, 7):
        for j in range(b.D):
            d = O.popcount(g[i] ^ g[j])
            assert d % 2 == 0
            if H[i, j] != 0.0:
                assert d in (0, 2, 4)


def test_count_difference_equals_popcount():
    rng = np.random.default_rng(3)
    for _ in range(2000):
        n_sp = int(rng.integers(2, 200))
        N = int(rng.integers(1, min(n_sp, 20) + 1))
        s1 = sorted(rng.choice(n_sp, N, replace=False).tolist())
        s2 = sorted(rng.choice(n_sp, N, replace=False).tolist())
        b1 = sum(1 << k for k in s1)
        b2 = sum(1 << k for k in s2)
        assert O.count_difference(s1, s2) == O.popcount(b1 ^ b2)


def test_low_word_prefilter_is_necessary():
    """Sec. 2.1: a popcount over the lowest 64 states never exceeds the full
    count, so screening on it cannot drop a connected pair."""
    rng = np.random.default_rng(5)
    for _ in range(2000):
        s1 = rng.choice(128, 8, replace=False)
        s2 = rng.choice(128, 8, replace=False)
        b1 = sum(1 << int(k) for k in s1)
        b2 = sum(1 << int(k) for k in s2)
        low = O.popcount((b1 ^ b2) & ((1 << 64) - 1))
        assert low <= O.popcount(b1 ^ b2)


def _running_totals(x):
    """Exclusive running totals by the standard library (itertools.accumulate
    over Python ints, so no overflow), a route independent of the oracle's
    loop."""
    return [0] + list(itertools.accumulate(int(v) for v in x))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 100, 1000, 4097])
def test_scan_against_running_totals(n):
    rng = np.random.default_rng(n)
    x = rng.integers(0, 5000, size=n)
    y = O.exclusive_scan(x)
    assert y[0] == 0 and len(y) == n + 1
    assert list(y) == _running_totals(x)
    assert all(int(y[k + 1]) - int(y[k]) == int(x[k]) for k in range(n))
    assert int(y[-1]) == int(x.sum())


def test_scan_empty_and_large_totals():
    assert list(O.exclusive_scan([])) == [0]
    x = np.full(3000, 2 ** 21, dtype=np.int64)          # total 6.3e9 > 2^32
    y = O.exclusive_scan(x)
    assert int(y[-1]) == 3000 * 2 ** 21
    assert list(y) == _running_totals(x)
