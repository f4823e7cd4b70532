"""Pins for the oracle's post-scoring selection (CPU only): segmented maximum and
top-k against numpy reductions / sorts, closed cases with ties and NaNs."""
import numpy as np

import oracle


def test_compound_best_matches_numpy_reduction():
    rng = np.random.default_rng(0)
    lens = rng.integers(1, 41, size=200)
    off = np.concatenate([[0], np.cumsum(lens)])
    s = np.round(rng.normal(6, 1.5, size=off[-1]), 1)        # rounding creates ties
    best, idx = oracle.compound_best(s, off)
    np.testing.assert_array_equal(best, np.maximum.reduceat(s, off[:-1]))
    for c in range(len(lens)):
        seg = s[off[c]:off[c + 1]]
        assert idx[c] == off[c] + int(np.argmax(seg))          # numpy's argmax: first maximum


def test_compound_best_edge_cases():
    s = np.array([np.nan, 2.0, 2.0, np.nan, -1.0])
    best, idx = oracle.compound_best(s, np.array([0, 1, 3, 4, 4, 5]))
    assert list(idx) == [-1, 1, -1, -1, 4]
    assert best[0] == -np.inf and best[1] == 2.0 and best[4] == -1.0


def test_top_k_matches_lexsort_and_is_a_prefix_of_the_full_order():
    rng = np.random.default_rng(1)
    v = np.round(rng.normal(size=3000), 2)
    full = oracle.top_k(v, len(v))
    want = np.lexsort((np.arange(len(v)), -v))                  # value desc, index asc
    np.testing.assert_array_equal(full, want)
    np.testing.assert_array_equal(oracle.top_k(v, 100), want[:100])


def test_top_k_nan_last_and_signed_zero_tie():
    v = np.array([np.nan, 0.0, -0.0, 5.0, np.nan, -3.0])
    assert list(oracle.top_k(v, 6)) == [3, 1, 2, 5, 0, 4]
