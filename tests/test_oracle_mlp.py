"""Pins of the FP64 network oracle: library special functions, finite
differences, the closed form of Adam's first steps and torch's bfloat16
conversion."""
import numpy as np
import scipy.stats
import torch

from oracle import mlp


def test_gelu_is_x_times_normal_cdf():
    x = np.linspace(-8, 8, 2001)
    assert np.max(np.abs(mlp.gelu(x) - x * scipy.stats.norm.cdf(x))) < 1e-15 * 8
    # gelu(x) - gelu(-x) = x because erf is odd
    assert np.max(np.abs(mlp.gelu(x) - mlp.gelu(-x) - x)) < 1e-14


def test_gelu_grad_central_difference():
    x = np.linspace(-6, 6, 241)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(4)
    widths = [12, 16, 16, 16, 16, 8]
    params = mlp.init(widths, 7)
    params = [(W, rng.normal(0, 0.1, size=b.shape)) for W, b in params]
    x = rng.normal(size=(5, 12))
    t = rng.normal(size=(5, 8))

    def loss(ps):
        y, _ = mlp.forward(ps, x)
        return mlp.mse(y, t)

    y, cache = mlp.forward(params, x)
    grads = mlp.backward(params, cache, y, t)
    h = 1e-6
    for layer in range(len(params)):
        for which in (0, 1):
            arr = params[layer][which]
            g = grads[layer][which]
            idx = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]
            for ix in idx:
                plus = [(W.copy(), b.copy()) for W, b in params]
                minus = [(W.copy(), b.copy()) for W, b in params]
                plus[layer][which][ix] += h
                minus[layer][which][ix] -= h
                fd = (loss(plus) - loss(minus)) / (2 * h)
                assert abs(fd - g[ix]) <= 1e-6 * max(1e-3, abs(fd)), (layer, which, ix)


def test_adam_closed_form_first_steps():
    """With zero moments, the bias-corrected first step is -lr g/(|g| + eps);
    under a constant gradient every later step is the same."""
    rng = np.random.default_rng(1)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    p1, m, v = mlp.adam_step(p, g, m, v, 1, lr, eps=eps)
    assert np.max(np.abs((p1 - p) - (-lr * g / (np.abs(g) + eps)))) < 1e-15
    p2, m, v = mlp.adam_step(p1, g, m, v, 2, lr, eps=eps)
    assert np.max(np.abs((p2 - p1) - (-lr * g / (np.abs(g) + eps)))) < 1e-14


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        [1.0 + 2.0**-8, 1.0 + 3 * 2.0**-8, -0.0, 0.0, 65504.0]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), want)
    assert mlp.bf16_round(1.0 + 2.0**-8) == 1.0          # tie to even
    assert mlp.bf16_round(1.0 + 3 * 2.0**-8) == 1.0 + 2.0**-6
