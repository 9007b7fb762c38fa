"""FP64 reference for the surrogate network: forward pass, hand-written reverse
mode, mean-squared-error loss and Adam.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product never
imports this module.

Network: x -> h_1 = gelu(x W_1 + b_1) -> ... -> h_L = gelu(h_{L-1} W_L + b_L)
-> y = h_L W_out + b_out, with gelu(u) = u * Phi(u) = 0.5 u (1 + erf(u/sqrt 2))
(the exact, erf-based form).  Weights are stored as W[in, out] (row-major
"in x out"), biases as b[out].  Loss = mean over batch and outputs of
(y - target)^2.  Adam (Kingma & Ba) with bias correction.

``round_hidden``: optional callable applied to every hidden activation and to
the network input before it enters a product, so that the reference can see
the same rounding points as a reduced-precision implementation when a test
asks for it.  With the default (None) everything is plain FP64.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

SQRT2 = np.sqrt(2.0)
INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)


def gelu(u):
    return 0.5 * u * (1.0 + erf(u / SQRT2))


def gelu_grad(u):
    """d/du [u Phi(u)] = Phi(u) + u phi(u)."""
    return 0.5 * (1.0 + erf(u / SQRT2)) + u * INV_SQRT_2PI * np.exp(-0.5 * u * u)


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64.  bfloat16 keeps the sign, the 8 exponent bits and the top 7
    mantissa bits of an IEEE binary32 value."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


def forward(params, x, round_hidden=None):
    """params: list of (W, b), hidden layers first, output layer last.
    Returns (y, cache) where cache holds what the backward pass needs."""
    rh = round_hidden or (lambda a: a)
    h = rh(np.asarray(x, dtype=np.float64))
    hs, us = [h], []
    for W, b in params[:-1]:
        u = h @ W + b
        h = rh(gelu(u))
        us.append(u)
        hs.append(h)
    W, b = params[-1]
    y = h @ W + b
    return y, (hs, us)


def mse(y, target):
    d = y - target
    return float(np.mean(d * d))


def backward(params, cache, y, target):
    """Gradients of the MSE loss w.r.t. every (W, b), by reverse mode."""
    hs, us = cache
    B, n_out = y.shape
    g = 2.0 * (y - target) / (B * n_out)        # dL/dy
    grads = [None] * len(params)
    W, _ = params[-1]
    grads[-1] = (hs[-1].T @ g, g.sum(axis=0))
    gh = g @ W.T                                   # dL/dh_L
    for layer in range(len(params) - 2, -1, -1):
        gu = gh * gelu_grad(us[layer])             # dL/du_layer
        grads[layer] = (hs[layer].T @ gu, gu.sum(axis=0))
        if layer > 0:
            gh = gu @ params[layer][0].T
    return grads


def adam_step(param, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (t >= 1); returns (param, m, v) as new arrays."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init(widths, seed):
    """Plain random initialisation (He-scaled normal weights, zero biases);
    used only for tests that need some network."""
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(widths[:-1], widths[1:]):
        params.append((rng.normal(0.0, np.sqrt(2.0 / a), size=(a, b)), np.zeros(b)))
    return params
