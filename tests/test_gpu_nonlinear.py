"""GPU parity of the nonlinear path (adi_set_laws, adi_set_pulse,
adi_set_iteration, adi_set_step_rule, adi_nl_step, adi_nl_run: the simple
iteration of eq. 12 and eq. 14 with the stop rule of eq. 13, step halving,
the pulsed source of eq. 2-4 and the step rule of Sec. 4) against the
oracle's nonlinear path, through the C ABI.

Step sequences (accepted steps, rejections, solves per half step, every
step's start time and size) must agree exactly; each case first checks that
the oracle's stop decisions were far from a tie, measured against how far
the two sides' fields may differ.  Fields agree to 1e-12 relative, except on
the case-study grid of Sec. 5 whose coating cells make the explicit half
steps stiff: there the bound is the rounding bound stiff_tol (see
test_nonlinear_emulation.py), computed from the run's own steps.  Both
sides are deterministic (the device's change norms are maxima, which do not
depend on the order of the atomic updates), so a case that passes keeps
passing."""
import math

import numpy as np
import pytest

import oracle
from helpers import gpu_available, rel_inf, tiny_spec
from paper_1912_03744_amd import workloads as W
from test_nonlinear_emulation import laws_of, nl_problem, stiff_tol

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-12


def gpu_problem(s, laws, T0):
    from paper_1912_03744_amd import native
    p = native.Problem.from_spec(s)
    p.set_laws(*laws)
    p.set_field(T0)
    return p


def seeded(nr, nz, seed=3):
    return W.production(seed, nr=nr, nz=nz).replace(h=(0.05, 0.1, 0.2, 0.1), t_inf=(0.0, 0.1, 0.0, 0.2))


@pytest.mark.parametrize("nr,nz", [(13, 31), (96, 240), (301, 699)])
def test_single_attempt(nr, nz):
    """One attempt at a fixed tau: the solves of each half step equal the
    oracle's and the field agrees to 1e-12 (grids of several chunks per lane
    and ragged ends)."""
    s = tiny_spec(nr, nz) if nr < 20 else seeded(nr, nz)
    laws = laws_of(s)
    P = nl_problem(s, laws)
    T0 = P.initial(0.5)
    tau = 0.02 if nr < 20 else 2e-3
    ok, want, its, chg = P.nl_step(T0, tau, 0.0, eps=1e-10, iter_max=40)
    assert ok and min(its) >= 3 and min(abs(c - 1e-10) / 1e-10 for c in chg) > 1e-2
    p = gpu_problem(s, laws, T0)
    p.set_iteration(1e-10, 40)
    acc, git, gchg = p.nl_step(tau)
    print("single attempt %dx%d: solves %s / oracle %s" % (nr, nz, git, its), flush=True)
    assert acc and git == its
    assert rel_inf(p.read_field(), want, P.active()) <= TOL


def test_constant_laws_equal_linear_paths():
    """Laws equal to constants: each half step stops at its second solve and
    the step equals the linear Peaceman-Rachford step, of the oracle and of
    the library's own linear path."""
    s = seeded(64, 160)
    z = np.zeros((5, 3))
    laws = (np.column_stack([s.k, z]), np.column_stack([s.rhoc, z]), np.column_stack([s.q, z]))
    P = oracle.Problem.from_spec(s)
    T0 = P.initial(0.3)
    want, _ = P.step(T0, "pr", 1e-3, 1)
    p = gpu_problem(s, laws, T0)
    p.set_iteration(1e-9, 10)
    acc, its, _ = p.nl_step(1e-3)
    assert acc and its == (2, 2)
    got = p.read_field()
    assert rel_inf(got, want, P.active()) <= TOL
    from paper_1912_03744_amd import native
    q = native.Problem.from_spec(s)
    q.set_field(T0)
    q.step(1e-3, 1)
    assert rel_inf(got, q.read_field(), P.active()) <= TOL


def test_iteration_limit_rejects_attempt():
    s = tiny_spec(9, 17)
    laws = laws_of(s, beta=2.0, gamma=1.0, chi=1.0)
    P = nl_problem(s, laws)
    T0 = P.initial(0.5)
    ok, _, its, _ = P.nl_step(T0, 0.5, 0.0, eps=1e-12, iter_max=2)
    assert not ok
    p = gpu_problem(s, laws, T0)
    p.set_iteration(1e-12, 2)
    acc, git, _ = p.nl_step(0.5)
    assert not acc and git == its
    act = P.active()
    assert np.array_equal(p.read_field()[act], T0[act])


@pytest.mark.parametrize("kind,nr,nz", [("rect", 10, 21), ("erf", 10, 21), ("erf", 96, 240)])
def test_adaptive_run(kind, nr, nz):
    """The time loop through a switch-on transition, the heating and the
    switch-off: every step agrees with the oracle's, the field to 1e-12."""
    s = tiny_spec(nr, nz) if nr < 20 else seeded(nr, nz)
    laws = laws_of(s)
    P = nl_problem(s, laws)
    T0 = P.initial(0.2)
    pulse = (0.02, 0.004, 2e-4, 4.0, 2.0)
    want = P.nl_run(T0, 0.0, 0.0062, kind=kind, pulse_args=pulse, eps=1e-10, iter_max=12, tau_trs_div=20.0,
                    tau_src_div=10.0, log_cap=4000)
    assert want["steps"] > 30 and want["min_margin"] > 1e-2
    p = gpu_problem(s, laws, T0)
    p.set_pulse(kind, *pulse)
    p.set_iteration(1e-10, 12)
    p.set_step_rule(20.0, 10.0)
    got = p.nl_run(0.0062, log_cap=4000)
    print("adaptive %s %dx%d: %d steps, %d rejected" % (kind, nr, nz, got["steps"], got["rejected"]), flush=True)
    for key in ("steps", "rejected", "solves_r", "solves_z"):
        assert got[key] == want[key], key
    assert np.array_equal(got["log"][:, 2:], want["log"][:, 2:])
    assert np.allclose(got["log"][:, :2], want["log"][:, :2], rtol=0, atol=1e-15)
    assert rel_inf(p.read_field(), want["T"], P.active()) <= TOL


def test_forced_halving():
    s = tiny_spec(8, 15)
    laws = laws_of(s, beta=1.5, gamma=0.8, chi=0.5)
    P = nl_problem(s, laws)
    T0 = P.initial(0.4)
    pulse = (0.1, 0.2, 1e-4, 4.0, 2.0)
    want = P.nl_run(T0, 0.0, 0.05, kind="const", pulse_args=pulse, eps=1e-6, iter_max=3, tau_src_div=1.0,
                    log_cap=1000)
    assert want["rejected"] > 0 and want["min_margin"] > 1e-3
    p = gpu_problem(s, laws, T0)
    p.set_pulse("const", *pulse)
    p.set_iteration(1e-6, 3)
    p.set_step_rule(1000.0, 1.0)
    got = p.nl_run(0.05, log_cap=1000)
    for key in ("steps", "rejected", "solves_r", "solves_z"):
        assert got[key] == want[key], key
    assert np.allclose(got["log"], want["log"], rtol=0, atol=1e-15)
    assert rel_inf(p.read_field(), want["T"], P.active()) <= TOL


def test_periodic_stop():
    s = tiny_spec(6, 11)
    laws = laws_of(s, beta=0.1, gamma=0.1, chi=0.05)
    P = nl_problem(s, laws)
    T0 = P.initial(0.0)
    pulse = (0.5, 0.1, 0.01, 4.0, 2.0)
    want = P.nl_run(T0, 0.0, 400.0, kind="erf", pulse_args=pulse, eps=1e-10, iter_max=12, tau_trs_div=4.0,
                    tau_src_div=5.0, periodic_tol=2e-3)
    assert want["periodic"] and want["min_margin"] > 1e-3
    p = gpu_problem(s, laws, T0)
    p.set_pulse("erf", *pulse)
    p.set_iteration(1e-10, 12)
    p.set_step_rule(4.0, 5.0, 2e-3)
    got = p.nl_run(400.0)
    assert got["periodic"]
    assert got["steps"] == want["steps"] and got["rejected"] == want["rejected"]
    assert abs(got["t"] - want["t"]) <= 1e-12
    assert rel_inf(p.read_field(), want["T"], P.active()) <= TOL


def _case_study_run(t0_field, t_end, scale=1.0, eps=1e-7):
    s = W.case_study(scale, scale)
    laws = W.case_study_laws()
    P = nl_problem(s, laws)
    T0 = P.initial(W.CASE_STUDY_T0) if t0_field is None else t0_field
    kw = dict(kind="erf", pulse_args=W.CASE_STUDY_PULSE, eps=eps, iter_max=10)
    want = P.nl_run(T0, 0.0, t_end, log_cap=100000, **kw)
    p = gpu_problem(s, laws, T0)
    p.set_pulse("erf", *W.CASE_STUDY_PULSE)
    p.set_iteration(eps, 10)
    got = p.nl_run(t_end, log_cap=100000)
    return s, P, want, got, p


def test_case_study_grid_first_transition():
    """The paper's case-study grid (1210 x 100 per-layer cells, Dirichlet top
    face) with the synthetic laws: the first 2e-5 of the switch-on
    transition (200 steps of t_trs/1000) against the oracle."""
    s, P, want, got, p = _case_study_run(None, 2e-5)
    lin = oracle.Problem.from_spec(s)
    tol = stiff_tol(lin, want["log"][:, 1], 1.5)
    err = rel_inf(p.read_field(), want["T"], P.active())
    print("case study 1210x100: %d steps, rel err %.2e, stiff bound %.2e" % (got["steps"], err, tol), flush=True)
    assert want["min_margin"] > 1e-3
    for key in ("steps", "rejected", "solves_r", "solves_z"):
        assert got[key] == want[key], key
    assert err <= tol


def test_case_study_scaled_grid_heating_pulse():
    """A tenth of the case-study grid in each direction (122 x 10), through
    the whole first heating pulse and into the cooling (0.012 of model time,
    about 2200 steps of both sizes)."""
    s, P, want, got, p = _case_study_run(None, 0.012, scale=0.1, eps=1e-7)
    lin = oracle.Problem.from_spec(s)
    tol = stiff_tol(lin, want["log"][:, 1], 1.5)
    err = rel_inf(p.read_field(), want["T"], P.active())
    print("case study 122x10: %d steps, rel err %.2e, stiff bound %.2e" % (got["steps"], err, tol), flush=True)
    assert want["min_margin"] > 1e-3
    for key in ("steps", "rejected", "solves_r", "solves_z"):
        assert got[key] == want[key], key
    assert err <= tol


def test_wait_bound_aborts_and_problem_recovers(monkeypatch):
    """The abort path of the kernel's grid-wide waits, forced from the host:
    with ADI_NL_WAIT_POLLS=0 the first wait that would poll aborts the run,
    every wave leaves at its next wait and adi_nl_run reports ADI_EDEVICE;
    with the default bound the same problem, its field set again, then runs
    to the oracle's result."""
    from paper_1912_03744_amd import native
    s = tiny_spec(10, 21)
    laws = laws_of(s)
    P = nl_problem(s, laws)
    T0 = P.initial(0.2)
    p = gpu_problem(s, laws, T0)
    p.set_iteration(1e-10, 12)
    monkeypatch.setenv("ADI_NL_WAIT_POLLS", "0")
    with pytest.raises(native.AdiError) as e:
        p.nl_run(2e-3)
    assert e.value.status == native.ADI_EDEVICE
    monkeypatch.delenv("ADI_NL_WAIT_POLLS")
    p.set_field(T0)
    want = P.nl_run(T0, 0.0, 2e-3, kind="const", eps=1e-10, iter_max=12)
    assert want["min_margin"] > 1e-3
    got = p.nl_run(2e-3)
    assert got["steps"] == want["steps"] and got["solves_r"] == want["solves_r"]
    assert rel_inf(p.read_field(), want["T"], P.active()) <= TOL


def test_state_and_argument_errors():
    from paper_1912_03744_amd import native
    s = tiny_spec(7, 12)
    p = native.Problem.from_spec(s)
    with pytest.raises(native.AdiError) as e:
        p.nl_step(0.1)
    assert e.value.status == native.ADI_ESTATE
    with pytest.raises(native.AdiError) as e:
        p.set_pulse("erf", 0.1, 0.2, 1e-4)      # t_src > t_per
    assert e.value.status == native.ADI_EINVAL
    with pytest.raises(native.AdiError) as e:
        p.set_iteration(1e-8, 65)
    assert e.value.status == native.ADI_EINVAL
    with pytest.raises(native.AdiError) as e:
        p.set_laws(np.full(20, np.nan), np.ones(20), np.zeros(20))
    assert e.value.status == native.ADI_ENONFINITE
