"""Pins of the oracle's sparsity pattern, prefix sum and state comparison.

* nnz from the brute-force pattern equals a class-pair count that never forms
  a state pair (Sec. 2.1 rule popcount <= 4 applied per species);
* every operator-generated entry has popcount(xor) in {0, 2, 4} (Sec. 2.1);
* count_difference (Listing 1 as a description) equals popcount of the xor;
* the serial counts-to-offsets recurrence (Sec. 2.2) equals the work-efficient
  up/down-sweep of Algorithm 1, restated here with the garbled loop bounds
  read as the standard Blelloch scan.
"""
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


def _blelloch(x):
    """Algorithm 1 of the paper, read as the standard work-efficient scan:
    pad to a power of two, up-sweep p = 0..log2(n)-1, clear the root, then
    down-sweep p = log2(n)-1..0.  Exclusive result of length len(x)."""
    n = 1
    while n < len(x):
        n *= 2
    y = np.zeros(n, dtype=object)
    y[:len(x)] = [int(v) for v in x]
    levels = n.bit_length() - 1
    for p in range(levels):
        for j in range(0, n, 2 ** (p + 1)):
            y[j + 2 ** (p + 1) - 1] = y[j + 2 ** p - 1] + y[j + 2 ** (p + 1) - 1]
    y[n - 1] = 0
    for p in range(levels - 1, -1, -1):
        for j in range(0, n, 2 ** (p + 1)):
            t = y[j + 2 ** p - 1]
            y[j + 2 ** p - 1] = y[j + 2 ** (p + 1) - 1]
            y[j + 2 ** (p + 1) - 1] = t + y[j + 2 ** (p + 1) - 1]
    return [int(v) for v in y[:len(x)]]


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 100, 1000, 4097])
def test_scan_recurrence_vs_blelloch(n):
    rng = np.random.default_rng(n)
    x = rng.integers(0, 5000, size=n)
    y = O.exclusive_scan(x)
    assert y[0] == 0 and len(y) == n + 1
    assert list(y[:-1]) == _blelloch(x)
    assert int(y[-1]) == int(x.sum())


def test_scan_empty_and_large_totals():
    assert list(O.exclusive_scan([])) == [0]
    x = np.full(3000, 2 ** 21, dtype=np.int64)          # total 6.3e9 > 2^32
    y = O.exclusive_scan(x)
    assert int(y[-1]) == 3000 * 2 ** 21
    assert list(y[:-1]) == _blelloch(x)
