"""GPU surrogate kernels (bf16 matrix cores, fp32 accumulation) against the
FP64 network oracle on the same bf16-rounded weights and inputs.

Tolerances: the GPU keeps hidden activations in bf16 (relative rounding up to
2^-8) and products in fp32.  Against a reference that rounds at the same
points the differences come from fp32 summation order and the occasional
one-ulp bf16 flip, so outputs must agree to 3e-3 relative l2 and element by
element to 1e-4 (64-wide network) or 2e-2 (256-wide) of the output scale,
which leaves no room for a misplaced tile or index; against the
plain FP64 reference, and for the gradients (whose backward signal is also
carried in bf16), each tensor must agree to 1e-2 relative l2 with cosine
similarity >= 0.999."""
import numpy as np
import pytest

from helpers import gpu_available
from oracle import mlp as O

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

WIDTHS = [12, 256, 256, 256, 256, 64]


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _cos(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def _setup(widths, seed, B):
    import torch
    from paper_1912_03744_amd import native
    net = native.MLP(widths, seed=seed)
    rng = np.random.default_rng(seed)
    p = net.params()
    p = p + rng.normal(0, 0.05, p.shape).astype(np.float32)  # non-zero biases too
    net.set_params(p)
    shift = rng.uniform(-1, 1, widths[0]).astype(np.float32)
    scale = rng.uniform(0.5, 2, widths[0]).astype(np.float32)
    net.set_scaling(shift, scale)
    x = rng.normal(size=(B, widths[0])).astype(np.float32)
    t = rng.normal(size=(B, widths[-1])).astype(np.float32)
    xd = torch.tensor(x, device="cuda")
    td = torch.tensor(t, device="cuda")
    # the oracle sees what the device computes with: bf16 weights, fp32 biases,
    # inputs encoded in fp32 then rounded to bf16
    ps = [(O.bf16_round(W), b.astype(np.float64)) for W, b in net.unflatten(p)]
    xe = O.bf16_round(((x - shift) * scale).astype(np.float32))
    return net, xd, td, ps, xe, t, p


@pytest.mark.parametrize("widths", [[12, 64, 64], WIDTHS, [12, 256, 256, 256, 256, 128]],
                         ids=["small", "surrogate64", "surrogate128"])
def test_forward_matches_oracle(widths):
    import torch
    net, xd, td, ps, xe, t, _ = _setup(widths, 1, 512)
    y = torch.empty(512, widths[-1], device="cuda")
    net.forward(xd, y)
    got = y.cpu().numpy().astype(np.float64)
    emu, _ = O.forward(ps, xe, round_hidden=O.bf16_round)
    plain, _ = O.forward(ps, xe)
    el = np.max(np.abs(got - emu)) / np.max(np.abs(emu))
    print("forward rel l2 vs rounded ref %.2e (elementwise %.2e), vs fp64 ref %.2e"
          % (_rel(got, emu), el, _rel(got, plain)), flush=True)
    assert _rel(got, emu) <= 3e-3
    assert _rel(got, plain) <= 1e-2 and _cos(got, plain) >= 0.999
    # element by element against the rounded reference: a wrong index in one
    # tile would move single outputs by O(1) of the output scale, far above a
    # bf16 rounding flip of one hidden value carried to the output
    assert el <= (1e-4 if widths[1] == 64 else 2e-2), el


@pytest.mark.parametrize("widths", [WIDTHS, [12, 256, 256, 256, 256, 128]], ids=["surrogate64", "surrogate128"])
def test_forward_large_batch_sampled_rows(widths):
    """A batch that gives every CU a workgroup of 256 rows takes the
    weight-resident layer kernels (smaller batches the tiled GEMM): 65,600
    rows (a ragged last workgroup) against the oracle on 1,024 sampled rows,
    the first and last included, and the tiled GEMM's output on the first
    4,096 rows as a batch of its own to the same tolerance."""
    import torch
    B = 65600
    net, xd, td, ps, xe, t, _ = _setup(widths, 3, B)
    y = torch.empty(B, widths[-1], device="cuda")
    net.forward(xd, y)
    got = y.cpu().numpy().astype(np.float64)
    rows = np.unique(np.concatenate([[0, B - 1], np.random.default_rng(3).choice(B, 1022, replace=False)]))
    emu, _ = O.forward(ps, xe[rows], round_hidden=O.bf16_round)
    plain, _ = O.forward(ps, xe[rows])
    el = np.max(np.abs(got[rows] - emu)) / np.max(np.abs(emu))
    print("large batch forward rel l2 vs rounded ref %.2e (elementwise %.2e), vs fp64 ref %.2e"
          % (_rel(got[rows], emu), el, _rel(got[rows], plain)), flush=True)
    assert _rel(got[rows], emu) <= 3e-3
    assert el <= 2e-2, el
    assert _rel(got[rows], plain) <= 1e-2 and _cos(got[rows], plain) >= 0.999
    y2 = torch.empty(4096, widths[-1], device="cuda")
    net.forward(xd[:4096].contiguous(), y2)
    small = y2.cpu().numpy().astype(np.float64)
    assert _rel(small, got[:4096]) <= 3e-3


@pytest.mark.parametrize("widths", [[12, 64, 64], WIDTHS], ids=["small", "surrogate"])
def test_gradients_match_oracle(widths):
    net, xd, td, ps, xe, t, _ = _setup(widths, 2, 1024)
    g, loss = net.gradients(xd, td)
    y, cache = O.forward(ps, xe, round_hidden=O.bf16_round)
    want = O.backward(ps, cache, y, t.astype(np.float64))
    assert abs(loss - O.mse(y, t)) <= 1e-3 * O.mse(y, t)
    for (gW, gb), (wW, wb) in zip(net.unflatten(g), want):
        for a, b in ((gW, wW), (gb, wb)):
            r, c = _rel(a.astype(np.float64), b), _cos(a.astype(np.float64), b)
            print("grad tensor %s rel %.2e cos %.6f" % (a.shape, r, c), flush=True)
            assert r <= 1e-2 and c >= 0.999


def test_adam_step_matches_oracle():
    """One training step equals Adam (closed form) applied to the device's
    own gradients of the same batch."""
    net, xd, td, ps, xe, t, p0 = _setup([12, 64, 64], 3, 256)
    g, _ = net.gradients(xd, td)
    net.set_params(p0)  # fresh optimiser state
    lr = 1e-3
    net.train_step(xd, td, lr)
    got = net.params().astype(np.float64)
    want, _, _ = O.adam_step(p0.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, lr)
    assert np.max(np.abs(got - want)) <= 1e-6


def test_training_reduces_loss():
    """A small smooth regression problem: the loss falls by 10x in 300 steps."""
    import torch
    from paper_1912_03744_amd import native
    rng = np.random.default_rng(7)
    net = native.MLP([4, 64, 64, 64], seed=11)
    net.set_scaling(np.zeros(4), np.ones(4))
    x = rng.uniform(-1, 1, size=(2048, 4)).astype(np.float32)
    w = rng.normal(size=(4, 64))
    t = np.tanh(x @ w).astype(np.float32) * 0.5
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    l0 = net.train_step(xd, td, 2e-3, want_loss=True)
    for _ in range(300):
        l1 = net.train_step(xd, td, 2e-3, want_loss=True)
    print("loss %.3e -> %.3e" % (l0, l1), flush=True)
    assert l1 < 0.1 * l0
