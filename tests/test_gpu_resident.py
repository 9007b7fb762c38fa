"""GPU parity of the LDS-resident layout (ADI_LAYOUT_RESIDENT: every run of
steps between energy checks in one launch of one workgroup holding the
right-hand side in LDS) against the oracle, element by element (relative
infinity norm over active cells <= 1e-12): the single layout of Fig. 1 over
its full 1000 steps in both schemes, grids at the kernel's limits with
non-zero ambient temperatures on every boundary class, energy checks between
the launches, continuation across calls, a switch of layout in mid-run, the
timing entry point and the size limits."""
import numpy as np
import pytest

import oracle
from helpers import gpu_available, rel_inf, run_gpu, run_oracle, tiny_spec
from paper_1912_03744_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-12


@pytest.mark.parametrize("scheme", ["lod", "pr"])
def test_single_layout_full_run(scheme):
    s = W.single_layout(scheme=scheme)
    print("resident single layout %s" % scheme, flush=True)
    P, want, _ = run_oracle(s, s.nsteps)
    p, got = run_gpu(s, s.nsteps, layout="resident")
    assert p.layout() == "resident"
    assert rel_inf(got, want, P.active()) <= TOL
    prof = p.profile(0, 64)
    wprof = P.profile(want, 0, 64)
    assert np.max(np.abs(prof - wprof)) <= TOL * np.max(np.abs(wprof))


@pytest.mark.parametrize("scheme", ["pr", "lod"])
@pytest.mark.parametrize("nr,nz", [(3, 3), (4, 5), (7, 12), (64, 160), (37, 91), (200, 13), (5, 256)])
def test_ambient_checks_continuation_and_switch(scheme, nr, nz):
    """Non-zero ambient temperatures on every face class, a Dirichlet class
    and the cut-out, a non-uniform start field, energy checks every 10 steps
    (check steps on the rows kernels, the runs between them resident), a
    continuation whose runs straddle the check pattern, then a switch to the
    rows layout that continues from the same state."""
    from paper_1912_03744_amd import native
    s = tiny_spec(scheme=scheme, dt=0.02).replace(nr=nr, nz=nz)
    P = oracle.Problem.from_spec(s)
    rng = np.random.default_rng(nr * 1000 + nz)
    T0 = np.where(P.active(), rng.uniform(0.0, 1.0, P.shape), 0.0)
    want1, _ = P.step(T0, s.scheme, s.dt, 23)
    want2, _ = P.step(want1, s.scheme, s.dt, 14)
    want3, _ = P.step(want2, s.scheme, s.dt, 5)
    print("resident ambient %s %dx%d" % (scheme, nr, nz), flush=True)
    p = native.Problem.from_spec(s)
    p.set_layout("resident")
    p.set_field(T0)
    p.set_check(10)
    p.step(s.dt, 23)
    assert rel_inf(p.read_field(), want1, P.active()) <= TOL
    p.step(s.dt, 14)
    assert rel_inf(p.read_field(), want2, P.active()) <= TOL
    p.set_layout("rows")
    p.step(s.dt, 5)
    assert rel_inf(p.read_field(), want3, P.active()) <= TOL


def test_timing_leaves_state_and_limits():
    from paper_1912_03744_amd import native
    s = W.single_layout(scheme="pr")
    P = oracle.Problem.from_spec(s)
    want, _ = P.step(P.initial(s.T0), "pr", s.dt, 20)
    p = native.Problem.from_spec(s)
    p.set_layout("resident")
    assert native.layout_shapes("resident", 0) == []
    p.step(s.dt, 10)
    ms, zero = p.time_sweeps(s.dt, 500)
    print("resident 64x160 pr: %.3f us per step" % (ms * 1e3), flush=True)
    assert ms > 0.0 and zero == 0.0
    p.step(s.dt, 10)
    assert rel_inf(p.read_field(), want, P.active()) <= TOL
    for nr, nz in ((513, 8), (8, 513), (100, 170), (2, 40)):
        q = native.Problem.from_spec(tiny_spec(nr=nr, nz=nz))
        with pytest.raises(native.AdiError) as e:
            q.set_layout("resident")
        assert e.value.status == native.ADI_EUNSUPPORTED
        assert q.layout() == "rows"
