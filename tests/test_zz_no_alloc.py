"""adi_mlp_forward_noalloc, the surrogate's forward pass for callers that
cannot allocate device memory, against adi_mlp_forward on the same network
and inputs: two calls in a row, the second with a smaller batch, each equal
bit for bit (the same products and epilogues; only where the activations
live differs).  The library's device allocations are counted through the
allocator hook: the no-alloc call must make none."""
import numpy as np
import pytest

from helpers import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

WIDTHS = [12, 256, 256, 256, 256, 64]


def test_forward_noalloc_matches_forward():
    import torch
    from paper_1912_03744_amd import native

    counts = {"alloc": 0}

    def alloc(n):
        counts["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(n)

    native.set_allocator(alloc, torch.cuda.caching_allocator_delete)
    try:
        net = native.MLP(WIDTHS, seed=7)
        rng = np.random.default_rng(7)
        p = net.params()
        net.set_params(p + rng.normal(0, 0.05, p.shape).astype(np.float32))
        net.set_scaling(rng.uniform(-1, 1, 12).astype(np.float32), rng.uniform(0.5, 2, 12).astype(np.float32))
        for B in (8192, 1088):   # the second call smaller than the first
            x = torch.tensor(rng.normal(size=(B, 12)).astype(np.float32), device="cuda")
            y0 = torch.full((B, 64), float("nan"), device="cuda")
            y1 = torch.full((B, 64), float("nan"), device="cuda")
            torch.cuda.synchronize()
            before = counts["alloc"]
            net.forward_noalloc(x, y0)
            torch.cuda.synchronize()
            print("noalloc forward: batch %d, %d device allocations" % (B, counts["alloc"] - before), flush=True)
            assert counts["alloc"] == before
            net.forward(x, y1)
            torch.cuda.synchronize()
            a, b = y0.cpu().numpy(), y1.cpu().numpy()
            assert np.isfinite(a).all()
            assert np.array_equal(a, b), np.max(np.abs(a - b))
        # a batch beyond the work area is refused before any device work
        x = torch.zeros((14592, 12), device="cuda")
        y = torch.zeros((14592, 64), device="cuda")
        with pytest.raises(native.AdiError) as e:
            net.forward_noalloc(x, y)
        assert e.value.status == native.ADI_EINVAL and "14528" in str(e.value)
        net.close()
    finally:
        native.set_allocator()
