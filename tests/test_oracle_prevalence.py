"""Pins for the prevalence / quantile reduction: numpy's default ('linear',
type 7) quantile is the same estimator, and prevalence is a plain ratio."""
import numpy as np

from oracle import prevalence as P


def test_type7_matches_numpy_quantile():
    rng = np.random.default_rng(3)
    for n in (1, 2, 5, 64, 257):
        x = rng.random(n)
        for p in (0.0, 0.1, 0.25, 0.5, 0.9, 1.0):
            assert abs(P.type7_quantile(x, p) - np.quantile(x, p)) <= 1e-15


def test_quantile_ties_and_order_invariance():
    x = [0.3, 0.1, 0.3, 0.2, 0.3]
    assert P.type7_quantile(x, 0.5) == 0.3
    assert P.type7_quantile(x[::-1], 0.1) == P.type7_quantile(x, 0.1)


def test_prevalence_ratio_and_empty_denominator():
    sums = np.zeros((2, 3, 3), dtype=np.int64)
    sums[0, 0] = [90, 10, 0]
    sums[0, 1] = [50, 25, 25]
    sums[1, 2] = [0, 0, 7]
    prev = P.prevalence(sums, 1, (0, 1))
    assert prev[0, 0] == 0.1 and prev[0, 1] == 25 / 75
    assert prev[1, 2] == 0.0 and prev[1, 0] == 0.0
    q = P.prevalence_quantiles(sums, 1, (0, 1), 2, 0, 3, (0.5,))
    assert q.shape == (1, 3, 1) and q.dtype == np.float32
    assert q[0, 0, 0] == np.float32(0.05)
