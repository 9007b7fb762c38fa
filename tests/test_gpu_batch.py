"""GPU parity of the ragged-batch path: every instance of a batch (own
geometry, materials and grid size) against the CPU oracle run alone, plus
batch-vs-single consistency, snapshot profiles and queue coverage."""
import numpy as np
import pytest

import oracle
from helpers import gpu_available, rel_inf
from paper_1912_03744_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]
TOL = 1e-12


def _oracle_run(s, nsteps):
    P = oracle.Problem.from_spec(s)
    T, _ = P.step(P.initial(s.T0), s.scheme, s.dt, nsteps)
    return P, T


@pytest.mark.parametrize("shape", [None, (4, 4, 2), (4, 1, 1)], ids=["default", "strips", "sweeps"])
@pytest.mark.parametrize("scheme", ["pr", "lod"])
def test_batch_instances_match_oracle(scheme, shape):
    """A stratified ragged batch (every size class, seeded designs) after 60
    steps with profiles every 20 steps, each instance against the oracle."""
    from paper_1912_03744_amd import native
    specs = W.ragged_batch(24, master_seed=5, scheme=scheme, dt=1e-3, nsteps=60)
    specs[3] = specs[3].replace(t_inf=(0.0, 0.3, -0.2, 0.1), T0=0.4)  # non-zero ambient and start
    b = native.Batch(specs, scheme=scheme)
    if shape:
        b.set_launch(*shape)
    b.step(1e-3, 60, snapshot_every=20, npts=64)
    prof = b.profiles()
    assert prof.shape == (24, 3, 64)
    print("batch %s: %s" % (scheme, b.info()), flush=True)
    for i, s in enumerate(specs):
        P, want = _oracle_run(s, 60)
        got = b.field(i)
        act = P.active()
        assert rel_inf(got, want, act) <= TOL, (i, s.nr, s.nz)
        assert np.all(got[~act] == 0.0)
        wp = P.profile(want, 0, 64)
        assert np.max(np.abs(prof[i, 2] - wp)) <= TOL * np.max(np.abs(wp))
        if i < 6:  # intermediate snapshot
            P2, w20 = _oracle_run(s, 20)
            wp20 = P2.profile(w20, 0, 64)
            assert np.max(np.abs(prof[i, 0] - wp20)) <= TOL * np.max(np.abs(wp20))


def test_batch_odd_sizes_and_launch_shapes():
    """Grid sizes between the compiled line shapes and tiny grids, under every
    batch launch shape; more instances than persistent workgroups."""
    from paper_1912_03744_amd import native
    rng = np.random.default_rng(1)
    base = W.ragged_batch(40, master_seed=9, nsteps=15)
    sizes = [(3, 3), (5, 7), (64, 160), (65, 161), (97, 241), (129, 321), (191, 479), (192, 480), (33, 400)]
    specs = [s.replace(nr=sizes[i % len(sizes)][0], nz=sizes[i % len(sizes)][1]) for i, s in enumerate(base)]
    want = [_oracle_run(s, 15) for s in specs]
    for shape in ((1, 4, 1), (2, 4, 2), (1, 8, 1), (2, 8, 1), (4, 4, 2), (4, 8, 1), (4, 1, 1)):
        b = native.Batch(specs)
        b.set_launch(*shape)
        b.step(1e-3, 15)
        for i in rng.choice(len(specs), 12, replace=False):
            P, w = want[i]
            assert rel_inf(b.field(int(i)), w, P.active()) <= TOL, (shape, i, specs[i].nr, specs[i].nz)


def test_batch_z_shapes_per_class():
    """Every compiled z shape of every z class of the batched sweep launches
    (odd sizes in each class and columns of each class's longest length)
    against the oracle; shapes out of range are refused."""
    from paper_1912_03744_amd import native
    classes = native.batch_zshapes()
    assert [c["max_rows"] for c in classes] == [192, 256, 320, 512]
    assert all(len(c["shapes"]) >= 2 for c in classes)
    sizes = [(5, 7), (64, 160), (33, 192), (96, 240), (40, 256), (7, 193), (128, 320), (61, 257),
             (192, 480), (65, 321), (9, 479), (100, 300)]
    base = W.ragged_batch(len(sizes), master_seed=13, nsteps=10)
    specs = [s.replace(nr=nr, nz=nz) for s, (nr, nz) in zip(base, sizes)]
    want = [_oracle_run(s, 10) for s in specs]
    b = native.Batch(specs)
    b.set_launch(4, 1, 1)
    for v in range(max(len(c["shapes"]) for c in classes)):
        for c, cl in enumerate(classes):
            b.set_zshape(c, v if v < len(cl["shapes"]) else 0)
        b.step(1e-3, 10)
        for i, s in enumerate(specs):
            P, w = want[i]
            assert rel_inf(b.field(i), w, P.active()) <= TOL, (v, i, s.nr, s.nz)
    for c, v in ((0, len(classes[0]["shapes"])), (4, 0), (-1, 0), (3, -1)):
        with pytest.raises(native.AdiError):
            b.set_zshape(c, v)
    b.close()


def test_batch_equals_single_instance_path():
    """Instance k of a batch reaches the single-instance GPU result (same
    method, different launch decomposition) to the parity tolerance."""
    from paper_1912_03744_amd import native
    specs = W.ragged_batch(8, master_seed=3, nsteps=40)
    b = native.Batch(specs)
    b.step(1e-3, 40)
    for i in (0, 5):
        p = native.Problem.from_spec(specs[i])
        p.step(1e-3, 40)
        single = p.read_field()
        act = ~np.isnan(single)
        assert rel_inf(b.field(i), single, act) <= TOL


def test_batch_errors():
    from paper_1912_03744_amd import native
    s = W.ragged_batch(2, master_seed=0)
    with pytest.raises(native.AdiError):
        native.Batch([s[0].replace(nr=193)])
    b = native.Batch(s)
    with pytest.raises(native.AdiError):
        b.set_launch(3, 4, 1)
    with pytest.raises(native.AdiError):
        b.step(-1.0, 10)


def test_batch_active_cells_and_timing():
    """The library's count of cells inside the domain equals the oracle's
    region maps, and the timed entry point leaves the same fields as a plain
    step call."""
    from paper_1912_03744_amd import native
    specs = W.ragged_batch(24, master_seed=5, nsteps=30)
    b = native.Batch(specs)
    want = sum(int(np.count_nonzero(oracle.Problem.from_spec(s).active())) for s in specs)
    assert b.active_cells() == want
    assert b.cells() == sum(s.nr * s.nz for s in specs)
    b.step(1e-3, 30)
    ref = [b.field(i) for i in (0, 7)]
    ms = b.time(1e-3, 30, 2)
    assert ms > 0.0
    for i, r in zip((0, 7), ref):
        assert np.array_equal(b.field(i), r)


def _host_threads():
    import os
    n = os.cpu_count() or 1
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, min(n, 16))


@pytest.mark.timeout(900)
def test_batch_full_size_stratified(tmp_path, monkeypatch):
    """The benchmark's batch: 4096 instances, 2000 steps, in the launch shape
    the autotuner picks; 16 instances per size class (64 in all, spread over
    the batch: the first, the last and evenly between) against the oracle run
    alone (field and terminal-face profile at t = 1 and 2)."""
    from paper_1912_03744_amd import autotune, native
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    specs = W.ragged_batch(4096, master_seed=0, scheme="pr", dt=1e-3, nsteps=2000)
    b = native.Batch(specs, scheme="pr")
    tuned = autotune.apply_batch(b, 1e-3, "pr", nsteps=50)
    print("batch tuned shape %s, z shapes %s" % (tuned["shape"], tuned.get("zshape")), flush=True)
    b.step(1e-3, 2000, snapshot_every=1000, npts=64)
    prof = b.profiles()
    picks = []
    for size in W.BATCH_SIZES:
        idx = [i for i, s in enumerate(specs) if (s.nr, s.nz) == size]
        sel = np.unique(np.linspace(0, len(idx) - 1, 16).round().astype(int))
        picks += [idx[k] for k in sel]
    assert len(picks) == 64
    threads = _host_threads()
    for i in picks:
        s = specs[i]
        P = oracle.Problem.from_spec(s)
        w1, _ = P.step_threads(P.initial(s.T0), "pr", 1e-3, 1000, threads)
        want, _ = P.step_threads(w1, "pr", 1e-3, 1000, threads)
        err = rel_inf(b.field(i), want, P.active())
        print("batch full size: instance %d (%dx%d) rel err %.2e" % (i, s.nr, s.nz, err), flush=True)
        assert err <= TOL, (i, s.nr, s.nz)
        for k, w in ((0, w1), (1, want)):
            wp = P.profile(w, 0, 64)
            assert np.max(np.abs(prof[i, k] - wp)) <= TOL * np.max(np.abs(wp)), (i, k)


def test_batch_sweeps_across_graph_segments():
    """Batched sweep launches over more steps than one captured graph holds
    (256): snapshots in the first and second graph and the final field
    against the oracle."""
    from paper_1912_03744_amd import native
    specs = W.ragged_batch(6, master_seed=21, scheme="pr", dt=1e-3, nsteps=300)
    b = native.Batch(specs, scheme="pr")
    b.set_launch(4, 1, 1)
    b.step(1e-3, 300, snapshot_every=100, npts=64)
    prof = b.profiles()
    assert prof.shape == (6, 3, 64)
    for i, s in enumerate(specs):
        P = oracle.Problem.from_spec(s)
        T = P.initial(s.T0)
        for k in range(3):
            T, _ = P.step(T, "pr", 1e-3, 100)
            wp = P.profile(T, 0, 64)
            assert np.max(np.abs(prof[i, k] - wp)) <= TOL * np.max(np.abs(wp)), (i, k)
        assert rel_inf(b.field(i), T, P.active()) <= TOL, i


def test_batch_profiles_into_device_buffer():
    """Snapshots written straight into a caller's device buffer (a torch
    tensor) equal the ones the batch keeps in its own buffer, and the host
    read of the last call returns the caller's buffer; npts must match."""
    import torch

    from paper_1912_03744_amd import native
    specs = W.ragged_batch(10, master_seed=4, scheme="pr", dt=1e-3, nsteps=40)
    for shape in ((4, 1, 1), (2, 8, 1)):
        b = native.Batch(specs, scheme="pr")
        b.set_launch(*shape)
        b.step(1e-3, 40, snapshot_every=10, npts=48)
        own = b.profiles()
        dev = torch.full((10, 4, 48), float("nan"), dtype=torch.float64, device="cuda")
        b.step(1e-3, 40, snapshot_every=10, npts=48, out=dev)
        b.sync()
        assert np.array_equal(dev.cpu().numpy(), own), shape
        assert np.array_equal(b.profiles(), own), shape
        with pytest.raises(native.AdiError):
            out = np.empty(own.size)
            native.check(native.lib().adi_batch_read_profiles(b._h, 64, native._ptr(out), out.size))
        P = oracle.Problem.from_spec(specs[7])
        T, _ = P.step(P.initial(specs[7].T0), "pr", 1e-3, 30)
        wp = P.profile(T, 0, 48)
        assert np.max(np.abs(own[7, 2] - wp)) <= TOL * np.max(np.abs(wp))
