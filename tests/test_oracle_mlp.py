"""Pins for the float64 surrogate-network reference: finite differences,
closed forms of GELU and the pinball loss, the first AdamW step, and
bfloat16 rounding against torch's conversion."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import mlp
from paper_1605_01421_amd import workloads as W


def test_gelu_closed_forms():
    z = np.linspace(-6, 6, 121)
    assert np.allclose(mlp.gelu(z), z * stats.norm.cdf(z), rtol=1e-14, atol=1e-300)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)


def test_pinball_values_and_quantile_minimiser():
    loss, g = mlp.pinball(np.array([[0.0, 1.0]]), np.array([[1.0, 0.0]]), (0.9,))
    assert loss == pytest.approx((0.9 * 1 + 0.1 * 1) / 2)
    assert np.allclose(g, [[-0.9 / 2, 0.1 / 2]])
    # the constant minimising the mean pinball loss is the empirical quantile
    rng = np.random.default_rng(0)
    t = rng.normal(size=999)
    grid = np.linspace(-3, 3, 6001)
    for q in (0.1, 0.5, 0.9):
        L = [np.mean(np.maximum(q * (t - c), (q - 1) * (t - c))) for c in grid]
        best = grid[int(np.argmin(L))]
        assert abs(best - np.quantile(t, q, method="inverted_cdf")) < 2e-3


def test_gradients_match_central_differences():
    dims = (3, 5, 4, 6)
    params = W.mlp_init(dims, seed=4)
    params = [(Wl, b + 0.1 * np.arange(len(b))) for Wl, b in params]
    rng = np.random.default_rng(1)
    X = rng.normal(size=(7, 3))
    Y0, _ = mlp.forward(params, X)
    T = Y0 + np.where(rng.random(Y0.shape) < 0.5, -1.0, 1.0) * (0.5 + rng.random(Y0.shape))
    probs = (0.1, 0.5, 0.9)
    loss, grads, _ = mlp.loss_and_grads(params, X, T, probs)
    h = 1e-6
    for l, (Wl, bl) in enumerate(params):
        for arr, g in ((Wl, grads[l][0]), (bl, grads[l][1])):
            num = np.zeros_like(arr)
            it = np.nditer(arr, flags=["multi_index"])
            for _ in it:
                i = it.multi_index
                old = arr[i]
                arr[i] = old + h
                lp = mlp.loss_and_grads(params, X, T, probs)[0]
                arr[i] = old - h
                lm = mlp.loss_and_grads(params, X, T, probs)[0]
                arr[i] = old
                num[i] = (lp - lm) / (2 * h)
            assert np.allclose(g, num, rtol=1e-6, atol=1e-9), l


def test_first_adamw_step_is_sign_step():
    params = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    grads = [(np.array([[0.3, -4.0]]), np.array([0.25]))]
    st = mlp.init_state(params)
    mlp.adamw_step(params, grads, st, lr=0.01, eps=1e-12, weight_decay=0.1)
    # m_hat = g, v_hat = g^2 on the first step -> update lr * (sign(g) + wd * w)
    assert np.allclose(params[0][0], [[1.0 - 0.01 * (1 + 0.1), -2.0 - 0.01 * (-1 + 0.1 * -2.0)]], rtol=1e-12)
    assert np.allclose(params[0][1], [0.5 - 0.01 * (1 + 0.1 * 0.5)], rtol=1e-12)


@pytest.mark.parametrize("beta1,beta2,eps", [(0.9, 0.999, 1e-8), (0.5, 0.7, 0.3)])
def test_adamw_constant_gradient_closed_form(beta1, beta2, eps):
    """With the same gradient g at every step, the bias-corrected moments are
    exactly m_hat = g and v_hat = g^2 at every t (that is what the
    corrections 1 - beta^t are for), so each step is the linear map
    w <- a w - c with a = 1 - lr wd and c = lr g / (|g| + eps), and
    w_t = a^t w_0 - c (1 - a^t) / (1 - a).  A wrong exponent in either
    correction, a missing eps or decay, breaks this at t >= 2."""
    lr, wd, T = 0.05, 0.2, 7
    g = np.array([[0.3, -4.0, 1e-3]])
    w0 = np.array([[1.0, -2.0, 0.7]])
    params = [(w0.copy(), np.array([0.0]))]
    st = mlp.init_state(params)
    a = 1.0 - lr * wd
    c = lr * g / (np.abs(g) + eps)
    for t in range(1, T + 1):
        mlp.adamw_step(params, [(g, np.array([0.0]))], st, lr=lr, beta1=beta1, beta2=beta2, eps=eps,
                       weight_decay=wd)
        want = a ** t * w0 - c * (1.0 - a ** t) / (1.0 - a)
        assert np.allclose(params[0][0], want, rtol=1e-11, atol=1e-14), t
        assert np.all(np.isfinite(params[0][1]))
    assert st["t"] == T


def test_adamw_moments_after_gradient_stops():
    """After t steps of gradient g and one step of gradient 0 (no decay), the
    corrected first moment is beta1 (1 - beta1^t) / (1 - beta1^(t+1)) g and the
    second beta2 (1 - beta2^t) / (1 - beta2^(t+1)) g^2: the step is
    lr m_hat / (sqrt(v_hat) + eps)."""
    b1, b2, eps, lr, t = 0.8, 0.95, 1e-3, 0.1, 4
    g = np.array([[2.0, -0.5]])
    params = [(np.zeros((1, 2)), np.array([0.0]))]
    st = mlp.init_state(params)
    for _ in range(t):
        mlp.adamw_step(params, [(g, np.array([0.0]))], st, lr=lr, beta1=b1, beta2=b2, eps=eps)
    before = params[0][0].copy()
    mlp.adamw_step(params, [(np.zeros_like(g), np.array([0.0]))], st, lr=lr, beta1=b1, beta2=b2, eps=eps)
    mh = b1 * (1 - b1 ** t) / (1 - b1 ** (t + 1)) * g
    vh = b2 * (1 - b2 ** t) / (1 - b2 ** (t + 1)) * g * g
    assert np.allclose(before - params[0][0], lr * mh / (np.sqrt(vh) + eps), rtol=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        1 + np.arange(1, 64) * 2.0 ** -9, [0.0, -0.0, 1e30, -3.5]])
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), want)
    assert mlp.bf16(np.array([1 + 2 ** -8]))[0] == 1.0  # tie to even


def test_ensemble_combine_closed_forms():
    """Members whose outputs form an arithmetic progression c + d k
    (k = 0..K-1) have mean c + d (K-1)/2 and sample standard deviation
    |d| sqrt(K (K+1) / 12); the de-standardisation scales both by y_std and
    shifts the mean by y_mean; one member disagrees by exactly 0, identical
    members by no more than the rounding of their mean."""
    rng = np.random.default_rng(9)
    B, N = 5, 7
    c = rng.normal(size=(B, N))
    d = rng.normal(size=(B, N))
    ymu, ysd = rng.normal(size=N), rng.uniform(0.5, 2.0, size=N)
    for K in (2, 3, 4, 7):
        P = np.stack([c + d * k for k in range(K)])
        mean, dis = mlp.ensemble_combine(P, ymu, ysd)
        assert np.allclose(mean, (c + d * (K - 1) / 2) * ysd + ymu, rtol=1e-13, atol=1e-13)
        want = (np.abs(d) * ysd * math.sqrt(K * (K + 1) / 12.0)).mean(axis=1)
        assert np.allclose(dis, want, rtol=1e-12)
    mean, dis = mlp.ensemble_combine(c[None], ymu, ysd)
    assert np.allclose(mean, c * ysd + ymu) and np.all(dis == 0.0)
    mean, dis = mlp.ensemble_combine(np.stack([c, c, c]), ymu, ysd)
    assert np.all(dis < 1e-15 * np.abs(c * ysd + ymu).max())  # only the rounding of the mean
