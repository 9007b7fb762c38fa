"""Device memory from the caller's allocator (adi_set_allocator): a problem,
a batch and a network allocated through PyTorch's caching allocator give the
same results as with hipMalloc, every block goes back to the allocator that
made it, and a hook changed while blocks are live still receives them."""
import numpy as np
import pytest

from helpers import gpu_available
from paper_1912_03744_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


class Counting:
    """Wraps torch's caching allocator and records the blocks it hands out."""

    def __init__(self):
        import torch
        self.torch = torch
        self.live = set()
        self.allocs = 0

    def alloc(self, n):
        p = self.torch.cuda.caching_allocator_alloc(n)
        self.live.add(p)
        self.allocs += 1
        return p

    def free(self, p):
        assert p in self.live
        self.live.remove(p)
        self.torch.cuda.caching_allocator_delete(p)


def _solve(native, spec, steps):
    p = native.Problem.from_spec(spec)
    p.step(spec.dt, steps)
    T = p.read_field()
    p.close()
    return T


def _batch(native, specs, steps):
    b = native.Batch(specs)
    b.set_launch(4, 1, 1)
    b.step(1e-3, steps, snapshot_every=steps, npts=64)
    out = [b.field(i) for i in range(len(specs))], b.profiles()
    b.close()
    return out


def test_allocator_hook_lifecycle():
    import torch
    from paper_1912_03744_amd import native
    torch.cuda.set_device(0)
    spec = W.single_layout(scheme="pr", nsteps=40)
    specs = W.ragged_batch(4, master_seed=7, nsteps=30)
    ref_T = _solve(native, spec, 40)
    ref_F, ref_P = _batch(native, specs, 30)
    hook = Counting()
    native.set_allocator(hook.alloc, hook.free)
    try:
        T = _solve(native, spec, 40)
        F, P = _batch(native, specs, 30)
        net = native.MLP([12, 64, 64], seed=3)
        x = torch.randn(128, 12, device="cuda")
        y = torch.empty(128, 64, device="cuda")
        net.forward(x, y)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
        assert hook.allocs > 0 and len(hook.live) > 0  # the network's blocks
        # blocks keep their owner when the hook changes while they are live
        native.set_allocator()
        net.close()
        assert not hook.live
    finally:
        native.set_allocator()
    act = ~np.isnan(ref_T)
    assert np.array_equal(T[act], ref_T[act])
    for a, b in zip(F, ref_F):
        assert np.array_equal(a, b)
    assert np.array_equal(P, ref_P)
