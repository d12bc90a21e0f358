"""Host-side logic of the surrogate: the disagreement threshold, the error
measure and the feature re-expression (no GPU)."""
import numpy as np

from paper_1605_01421_amd import surrogate as S


def test_choose_threshold_largest_prefix_within_eps():
    dis = np.array([0.4, 0.1, 0.3, 0.2])
    err = np.array([5.0, 1.0, 5.0, 1.0])
    # by disagreement: 0.1 (1), 0.2 (1), 0.3 (5), 0.4 (5); running means 1, 1, 7/3, 3
    assert S.choose_threshold(dis, err, 2.0) == 0.2
    assert S.choose_threshold(dis, err, 7.0 / 3.0) == 0.3
    assert S.choose_threshold(dis, err, 3.0) == 0.4
    assert S.choose_threshold(dis, err, 0.5) == -np.inf


def test_accepted_mean_error_respects_eps():
    rng = np.random.default_rng(1)
    dis = rng.random(500)
    err = dis * 2 + rng.random(500) * 0.5
    eps = float(np.quantile(err, 0.3))
    th = S.choose_threshold(dis, err, eps)
    acc = dis <= th
    assert acc.any() and err[acc].mean() <= eps
    # one more set would break it (the threshold is the largest such)
    nxt = np.sort(dis[~acc])[0]
    assert err[dis <= nxt].mean() > eps


def test_mean_abs_error_and_transform():
    a = np.zeros((3, 52, 3))
    b = np.ones((3, 52, 3)) * np.array([1.0, 2.0, 3.0])[:, None, None]
    assert np.allclose(S.mean_abs_error(a, b), [1.0, 2.0, 3.0])
    X = np.array([[0, 0.16, 0, 0.08, 0.01, 4.0, 0.5, 7.0], [1, 0, 0.02, 0.1, 0.02, 3.0, 0.4, 6.0]])
    Z = S.Ensemble._transform(X)
    assert Z.shape == (2, 8)
    assert np.allclose(Z[:, 1], X[:, 1] / X[:, 3]) and np.allclose(Z[:, 2], X[:, 2] / X[:, 3])
    assert np.allclose(Z[:, 3], np.log(X[:, 3])) and np.allclose(Z[:, 4], np.log(X[:, 4]))
    assert np.array_equal(Z[:, [0, 5, 6, 7]], X[:, [0, 5, 6, 7]])


def test_combined_threshold_keeps_combined_error_at_most_ssa():
    """The combined threshold accepts, by increasing disagreement, the
    longest prefix whose network errors do not exceed the SSA's in sum: the
    combined error on those sets is then <= the SSA's, and one more set would
    break it."""
    dis = np.array([0.1, 0.2, 0.3, 0.4, 0.5])
    e_nn = np.array([1.0, 3.0, 1.0, 9.0, 0.0])
    e_ssa = np.array([2.0, 2.0, 2.0, 2.0, 2.0])
    # running sums of e_nn - e_ssa: -1, 0, -1, 6, 4
    assert S.choose_threshold_combined(dis, e_nn, e_ssa) == 0.3
    assert S.choose_threshold_combined(dis, e_nn + 5, e_ssa) == -np.inf
    rng = np.random.default_rng(4)
    dis = rng.random(400)
    e_ssa = 1.0 + 0.2 * rng.random(400)
    e_nn = 2.0 * dis + 0.3 * rng.random(400)
    th = S.choose_threshold_combined(dis, e_nn, e_ssa)
    acc = dis <= th
    comb = np.where(acc, e_nn, e_ssa)
    assert acc.any() and comb.mean() <= e_ssa.mean() + 1e-12
    nxt = np.sort(dis[~acc])
    assert all(np.where(dis <= x, e_nn, e_ssa).mean() > e_ssa.mean() for x in nxt[:1])
