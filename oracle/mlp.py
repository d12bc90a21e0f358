"""Float64 reference for the surrogate network (TEST INFRASTRUCTURE ONLY).

A multilayer perceptron maps the 8 features of a parameter set to the
weekly prevalence quantiles an SSA ensemble produces:

    Z_l = A_{l-1} W_l^T + b_l,   A_l = GELU(Z_l) for hidden layers,
    Y   = Z_L (no activation on the output layer),

GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 (the exact form), trained on
the pinball (quantile) loss averaged over the batch and outputs,

    L = mean_{b,j} max(q_j (t - y), (q_j - 1) (t - y)),

where output j estimates the quantile q_j = probs[j mod len(probs)].  The
sub-gradient used at t == y is q_j - 1 (the y > t branch is taken for
t - y <= 0).  Optimiser: AdamW (decoupled weight decay, Loshchilov & Hutter).

``round_bf16`` lets the reference round activations and back-propagated
gradients to bfloat16 at the same points as a mixed-precision implementation
(inputs, hidden activations, output gradient and hidden-layer gradients
before they enter a product), so a GPU implementation can be compared at
the precision it computes in.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float64/float32 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(f), f, out).astype(np.float64)


def gelu(z):
    # Phi(z) = erfc(-z / sqrt 2) / 2, the form without cancellation for z < 0
    return 0.5 * z * erfc(-z / SQRT2)


def gelu_grad(z):
    return 0.5 * erfc(-z / SQRT2) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def forward(params, X, round_bf16=False):
    """params: list of (W (out, in), b (out,)).  Returns (Y, cache)."""
    A = bf16(X) if round_bf16 else np.asarray(X, dtype=np.float64)
    acts, zs = [A], []
    for l, (W, b) in enumerate(params):
        Z = A @ W.T + b
        zs.append(Z)
        if l + 1 < len(params):
            A = gelu(Z)
            if round_bf16:
                A = bf16(A)
            acts.append(A)
    return zs[-1], (acts, zs)


def pinball(Y, T, probs):
    """Mean pinball loss and its gradient with respect to Y."""
    q = np.resize(np.asarray(probs, dtype=np.float64), Y.shape[1])[None, :]
    d = T - Y
    loss = np.where(d > 0, q * d, (q - 1.0) * d)
    grad = np.where(d > 0, -q, 1.0 - q) / Y.size
    return loss.mean(), grad


def backward(params, cache, dY, round_bf16=False):
    """Gradients [(dW, db)] of the loss whose gradient wrt the output is dY."""
    acts, zs = cache
    grads = [None] * len(params)
    dZ = bf16(dY) if round_bf16 else dY
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        grads[l] = (dZ.T @ acts[l], dZ.sum(axis=0))
        if l > 0:
            dA = dZ @ W
            dZ = dA * gelu_grad(zs[l - 1])
            if round_bf16:
                dZ = bf16(dZ)
    return grads


def loss_and_grads(params, X, T, probs, round_bf16=False):
    Y, cache = forward(params, X, round_bf16)
    loss, dY = pinball(Y, T, probs)
    return loss, backward(params, cache, dY, round_bf16), Y


def adamw_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One AdamW update in place.  state = {'t': int, 'm': [...], 'v': [...]}."""
    state["t"] += 1
    t = state["t"]
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m = state["m"][2 * i + j]
            v = state["v"][2 * i + j]
            m *= beta1
            m += (1.0 - beta1) * g
            v *= beta2
            v += (1.0 - beta2) * g * g
            mhat = m / (1.0 - beta1 ** t)
            vhat = v / (1.0 - beta2 ** t)
            p -= lr * (mhat / (np.sqrt(vhat) + eps) + weight_decay * p)


def init_state(params):
    return {"t": 0, "m": [np.zeros_like(a) for W, b in params for a in (W, b)],
            "v": [np.zeros_like(a) for W, b in params for a in (W, b)]}


def ensemble_combine(P, y_mean, y_std):
    """The ensemble's answer from its members' standardised outputs P
    (members, B, N): y = P * y_std + y_mean per member, the mean over the
    members (B, N) and the disagreement (B,) = mean over the outputs of the
    members' sample standard deviation (divisor members - 1; 0 for one
    member).  Float64, written out from the definition."""
    P = np.asarray(P, dtype=np.float64)
    K = P.shape[0]
    y = P * np.asarray(y_std, dtype=np.float64)[None, None, :] + np.asarray(y_mean, dtype=np.float64)[None, None, :]
    mean = y.sum(axis=0) / K
    if K > 1:
        sd = np.sqrt(((y - mean[None]) ** 2).sum(axis=0) / (K - 1))
    else:
        sd = np.zeros_like(mean)
    return mean, sd.mean(axis=1)
