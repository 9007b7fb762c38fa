"""Pins of the oracle's nonlinear path: the simple (Picard) iteration of
Sec. 3 (eq. 12-14) with its stop rule (eq. 13) and time-step halving, the
pulsed source of Sec. 2 (eq. 2-4) and the step-size rule of Sec. 4.  Each
pin comes from outside the oracle: the linear path (constant laws), a scalar
recurrence solved by a library root finder, the Kirchhoff transform of the
steady nonlinear problem, closed forms of the pulse, and the defining
properties of the halving and step rules.
"""
import math

import numpy as np
import pytest
import scipy.optimize

import oracle
from paper_1912_03744_amd import workloads as W

PULSE = (0.1, 0.01, 1e-4, 4.0, 2.0)  # t_per, t_src, t_trs, xi, zeta of the case study (Sec. 5, Fig. 2)


def tiny_spec(nr=7, nz=12):
    return W.Spec(r0=1.0, r1=1.6, r2=2.3, rmax=2.6, z0=3.1, zmax=4.4, ztop=5.0, nr=nr, nz=nz,
                  h=(0.3, 0.2, math.inf, 0.15), t_inf=(0.4, -0.3, 0.25, 0.1),
                  k=(0.8, 0.07, 1.3, 0.2, 2.1), rhoc=(1.1, 0.6, 1.7, 0.9, 1.3),
                  q=(0.2, 0.0, 1.5, 0.3, 0.1))


def nl_problem(s):
    return oracle.NonlinearProblem((s.r0, s.r1, s.r2, s.rmax, s.z0, s.zmax, s.ztop), s.nr, s.nz,
                                   s.h, s.t_inf, s.k, s.rhoc, s.q, s.r_faces, s.z_faces)


def mild_laws(s, beta=0.3, gamma=0.2, chi=0.1):
    """Conductivity k (1 + beta T), capacity rho c (1 + gamma T^2), source
    q (1 + chi T): every coefficient positive for T >= 0."""
    lam = np.zeros((5, 4))
    cap = np.zeros((5, 4))
    src = np.zeros((5, 4))
    lam[:, 0], lam[:, 1] = s.k, np.asarray(s.k) * beta
    cap[:, 0], cap[:, 2] = s.rhoc, np.asarray(s.rhoc) * gamma
    src[:, 0], src[:, 1] = s.q, np.asarray(s.q) * chi
    return lam, cap, src


# ------------------------------------------------ the pulse (eq. 2-4) --

def test_rectangular_pulse_closed_form():
    """u(t) of eq. 3 is 1 for the first t_src of every period and 0 after."""
    tper, tsrc = PULSE[0], PULSE[1]
    for t in (0.0, 0.004, 0.0099, 0.0101, 0.05, 0.0999, 0.1, 0.103, 0.2 + 0.011, 3.004, 3.02):
        ph = t - math.floor(t / tper + 1e-12) * tper
        want = 1.0 if ph < tsrc - 1e-12 else 0.0
        assert oracle.pulse("rect", t, *PULSE) == want, t


def test_smoothed_pulse_properties():
    """v(t) of eq. 4: one half at the middle of every transition (erf(0) = 0),
    within erfc(xi) of u(t) outside the transitions, periodic, and its
    integral over a period equals t_src (the switch-off edge is the
    switch-on edge shifted by t_src)."""
    tper, tsrc, ttrs = PULSE[:3]
    for n in (0, 1, 7, 40):
        on = n * tper + ttrs / 2
        off = n * tper + tsrc + ttrs / 2
        # the rounding of t (about 1e-16 t) moves the erf argument by
        # xi zeta/t_trs times that
        tol = 1e-13 + 0.6 * PULSE[3] * PULSE[4] / ttrs * 2.3e-16 * off
        assert abs(oracle.pulse("erf", on, *PULSE) - 0.5) < tol
        assert abs(oracle.pulse("erf", off, *PULSE) - 0.5) < tol
    tail = math.erfc(PULSE[3])
    for t in (0.003, 0.0061, 0.03, 0.0805, 1.005, 2.3):
        assert abs(oracle.pulse("erf", t, *PULSE) - oracle.pulse("rect", t, *PULSE)) <= tail
    for t in (0.00003, 0.01007, 0.0504):
        assert abs(oracle.pulse("erf", t + 3 * tper, *PULSE) - oracle.pulse("erf", t, *PULSE)) < 1e-9
    # integral over one period by the midpoint rule on a fine grid
    n = 200000
    ts = (np.arange(n) + 0.5) * (tper / n) + 2 * tper
    vals = np.array([oracle.pulse("erf", t, *PULSE) for t in ts[::50]])
    # coarse check on the sparse sample, then the transitions finely
    assert abs(vals.mean() * tper - tsrc) < 2 * tper / len(vals)
    fine = (np.arange(20000) + 0.5) * (4 * ttrs / 20000)
    edge_on = np.array([oracle.pulse("erf", 2 * tper - ttrs + x, *PULSE) for x in fine])
    edge_off = np.array([oracle.pulse("erf", 2 * tper + tsrc - ttrs + x, *PULSE) for x in fine])
    # rise + fall integrate to the length of the window exactly (symmetry)
    assert abs((edge_on + edge_off).mean() - 1.0) < 1e-9


def test_constant_pulse():
    assert oracle.pulse("const", 0.37, *PULSE) == 1.0


# ------------------------------- the iteration reduces to the linear path --

def test_constant_laws_reproduce_linear_step():
    """With temperature-independent laws the iterate after the first solve
    is already the linear half step, so the second solve repeats it exactly
    and the stop rule of eq. 13 ends each half step after 2 solves; the step
    equals the Peaceman-Rachford step of eq. 8-9 bit for bit."""
    s = tiny_spec()
    P = nl_problem(s)
    P.set_constant_laws(s.k, s.rhoc, s.q)
    rng = np.random.default_rng(3)
    T = np.where(P.active(), rng.uniform(0, 1, P.shape), 0.0)
    for dt in (0.01, 0.3):
        want, _ = P.step(T, "pr", dt, 1)
        ok, got, it, chg = P.nl_step(T, dt, 0.0, eps=1e-12)
        assert ok and it == (2, 2) and chg[0] == 0.0 and chg[1] == 0.0
        assert np.array_equal(got, want)
    # several steps, with the constant pulse
    Tn = T
    for k in range(5):
        ok, Tn, it, _ = P.nl_step(Tn, 0.02, 0.02 * k, eps=1e-12)
        assert ok
    want, _ = P.step(T, "pr", 0.02, 5)
    assert np.array_equal(Tn, want)


def test_uniform_field_scalar_recurrence():
    """One material, insulated faces, uniform start: every cell follows the
    scalar recurrence C(Tb) (Tb - T) = (tau/2) X(Tb) p and C(Tb) (Th - Tb) =
    (tau/2) X(Tb) p, with p taken at t + tau/2.  Tb is found here by a
    library root finder; the iteration converges to it."""
    s = W.single_layout(nr=6, nz=14).replace(h=(0.0,) * 4, k=(0.6,) * 5, rhoc=(1.3,) * 5, q=(0.8,) * 5)
    P = nl_problem(s)
    cap = np.tile([1.3, 0.0, 0.45, 0.0], (5, 1))
    src = np.tile([0.8, -0.2, 0.0, 0.05], (5, 1))
    lam = np.tile([0.6, 0.5, 0.0, 0.0], (5, 1))
    P.set_laws(lam, cap, src)
    C = lambda T: 1.3 + 0.45 * T * T
    X = lambda T: 0.8 - 0.2 * T + 0.05 * T ** 3
    T = P.initial(0.5)
    act = P.active()
    Tv, t, tau = 0.5, 0.0, 2e-4
    for k in range(12):
        p = oracle.pulse("erf", t + tau / 2, *PULSE)
        Tb = scipy.optimize.brentq(lambda y: C(y) * (y - Tv) - 0.5 * tau * X(y) * p, Tv - 1, Tv + 1, xtol=1e-15)
        Th = Tb + 0.5 * tau * X(Tb) * p / C(Tb)
        ok, T, it, _ = P.nl_step(T, tau, t, kind="erf", pulse_args=PULSE, eps=1e-15, iter_max=50)
        assert ok
        assert np.max(np.abs(T[act] - Th)) <= 1e-13 * abs(Th), k
        Tv, t = Th, t + tau


# ------------------------- face conductivity of the iteration (Kirchhoff) --

def test_face_conductivity_kirchhoff_identity():
    """With laws lambda_m(T) = k_m (1 + beta T) (one beta for every region)
    the Kirchhoff variable U = T + beta T^2/2 turns the flux through every
    face between two cells into the linear flux of U: with each side's
    conductivity taken at the mean face temperature, the series conductance
    is (1 + beta T_f) times the linear one and (1 + beta T_f)(T_b - T_a) =
    U_b - U_a exactly.  So on every cell without a boundary face the
    nonlinear operators applied to T equal the linear operators (constant
    k_m) applied to U, to rounding; a conductivity taken from one cell only
    breaks this.  Checked on the masked layered grid, all regions, both
    directions, non-uniform faces."""
    beta = 0.7
    s = tiny_spec(nr=11, nz=17)
    rf = W.layer_aligned_faces((0.0, s.r0, s.r1, s.r2, s.rmax), (4, 2, 3, 2))
    zf = W.layer_aligned_faces((0.0, s.z0, s.zmax, s.ztop), (9, 5, 3))
    s = s.replace(r_faces=rf, z_faces=zf)
    P = nl_problem(s)
    lam = np.column_stack([s.k, np.asarray(s.k) * beta, np.zeros(5), np.zeros(5)])
    P.set_laws(lam, np.tile([1.0, 0, 0, 0], (5, 1)), np.zeros((5, 4)))
    rng = np.random.default_rng(4)
    T = np.where(P.active(), rng.uniform(0.0, 3.0, P.shape), 0.0)
    U = T + beta * T * T / 2
    ar, az = P.nl_apply(T, T)
    lin_r, lin_z = P.apply(U)
    b_r, b_z = P.apply(np.zeros(P.shape))
    m = P.region_map()
    act = m != oracle.MASKED
    # cells whose r (z) faces all lie between two cells of the domain
    inner_r = act.copy()
    inner_r[:, -1] = False
    inner_r[:, 1:] &= act[:, :-1]
    inner_r[:, :-1] &= act[:, 1:]
    inner_z = act.copy()
    inner_z[0, :] = False
    inner_z[-1, :] = False
    inner_z[1:, :] &= act[:-1, :]
    inner_z[:-1, :] &= act[1:, :]
    assert inner_r.sum() > 50 and inner_z.sum() > 50
    assert np.all(b_r[inner_r] == 0) and np.all(b_z[inner_z] == 0)
    scale = np.max(np.abs(lin_r[inner_r])) + np.max(np.abs(lin_z[inner_z]))
    assert np.max(np.abs(ar[inner_r] - lin_r[inner_r])) <= 1e-13 * scale
    assert np.max(np.abs(az[inner_z] - lin_z[inner_z])) <= 1e-13 * scale
    # the laws are taken from F, not from the field they act on
    ar2, _ = P.nl_apply(np.zeros(P.shape), T)
    assert np.max(np.abs(ar2 - P.apply(T)[0])) <= 1e-13 * np.max(np.abs(ar2))


# -------------------------------- halving and the step rule (Sec. 3-4) --

def _steep_problem():
    s = tiny_spec(nr=9, nz=14).replace(h=(0.0, 0.5, 0.4, 0.2), t_inf=(0.0,) * 4)
    P = nl_problem(s)
    lam, cap, src = mild_laws(s, beta=2.0, gamma=0.5, chi=0.5)
    P.set_laws(lam, cap, src)
    rng = np.random.default_rng(11)
    T = np.where(P.active(), rng.uniform(0.0, 2.0, P.shape), 0.0)
    return P, T


def test_step_halving_until_the_iteration_stops():
    """When the iteration does not stop within iter_max solves the step is
    retried with tau/2 (end of Sec. 3): the accepted step is the first of
    tau0, tau0/2, tau0/4, ... whose two iterations both stop, and each
    rejection is counted."""
    P, T = _steep_problem()
    tau0 = PULSE[1] / 100 * 50  # the rule's step for a constant source with t_src = 0.5
    args = (0.1, 0.5, 1e-4, 4.0, 2.0)
    res = P.nl_run(T, 0.0, 10.0, kind="const", pulse_args=args, eps=1e-9, iter_max=4, max_steps=1,
                   log_cap=1)
    assert res["steps"] == 1 and res["rejected"] >= 2
    tau = res["log"][0, 1]
    k = res["rejected"]
    assert tau == tau0 / 2 ** k
    ok, got, it, _ = P.nl_step(T, tau, 0.0, eps=1e-9, iter_max=4)
    assert ok and np.array_equal(got, res["T"])
    assert tuple(res["log"][0, 2:]) == it
    for j in range(k):
        ok, _, _, _ = P.nl_step(T, tau0 / 2 ** j, 0.0, eps=1e-9, iter_max=4)
        assert not ok, j


def test_stop_rule_first_change_below_eps():
    """Eq. 13: a half step stops at the first solve whose change from the
    previous iterate is below eps.  Limiting the solves to j < k makes the
    step fail with the j-th change at or above eps; with k solves it passes
    with the k-th change below eps."""
    P, T = _steep_problem()
    for eps in (1e-6, 3e-9, 1e-11):
        ok, _, it, chg = P.nl_step(T, 0.02, 0.0, eps=eps, iter_max=60)
        assert ok and chg[0] < eps and chg[1] < eps
        k = it[0]
        assert k >= 3
        for j in range(1, k):
            ok, _, itj, chgj = P.nl_step(T, 0.02, 0.0, eps=eps, iter_max=j)
            assert not ok and itj[0] == -1 and chgj[0] >= eps, (eps, j)


def test_single_solve_limit_forces_halving():
    """With at most one solve per half step a step is accepted only once its
    change T^1 - T^0 itself is below eps: the step is halved repeatedly."""
    P, T = _steep_problem()
    args = (0.1, 0.5, 1e-4, 4.0, 2.0)
    res = P.nl_run(T, 0.0, 10.0, kind="const", pulse_args=args, eps=1e-3, iter_max=1, max_steps=1,
                   log_cap=1)
    assert res["rejected"] >= 4 and res["log"][0, 2] == 1 and res["log"][0, 3] == 1
    assert np.max(np.abs(res["T"] - T)) < 2e-3


def test_step_size_rule_over_switching():
    """Sec. 4: inside a transition of the source (the first t_trs after each
    switch-on or switch-off) the step is t_trs/1000, elsewhere t_src/100;
    steps end on the switch points and transition ends, and add up to t_end
    exactly.  Mild laws, so that no step is halved."""
    s = tiny_spec(nr=5, nz=8)
    P = nl_problem(s)
    lam, cap, src = mild_laws(s, beta=0.05, gamma=0.05, chi=0.05)
    P.set_laws(lam, cap, src)
    T = P.initial(0.2)
    t_end = 0.0125
    res = P.nl_run(T, 0.0, t_end, kind="erf", pulse_args=PULSE, eps=1e-8, iter_max=20, log_cap=10000)
    assert res["rejected"] == 0
    log = res["log"]
    assert abs(res["t"] - t_end) <= 1e-15
    ts, taus = log[:, 0], log[:, 1]
    ttrs, tsrc = PULSE[2], PULSE[1]
    fine = (ts < ttrs - 1e-12) | ((ts >= tsrc - 1e-12) & (ts < tsrc + ttrs - 1e-12))
    assert np.all(np.abs(taus[fine] - ttrs / 1000) <= 1e-9 * ttrs / 1000)
    coarse = ~fine
    # coarse steps take t_src/100 unless cut at the next switch point or t_end
    cut = np.abs(taus[coarse] - tsrc / 100) > 1e-12 * tsrc
    ends = ts[coarse][cut] + taus[coarse][cut]
    for e in ends:
        assert min(abs(e - b) for b in (ttrs, tsrc, tsrc + ttrs, t_end)) < 1e-15, e
    for b in (ttrs, tsrc, tsrc + ttrs):
        assert np.min(np.abs(ts - b)) < 1e-15, b
    assert np.sum(fine) >= 2000
    assert abs(np.sum(taus) - t_end) < 1e-14


def test_periodic_regime_stop():
    """The run stops at the first period start at which the field differs
    from the previous period start by less than the tolerance: at once for a
    field that no longer changes, and, for a pulsed heater cooled through a
    film, at a period start after which one more period changes the field
    by less than the tolerance (up to the contraction of a period)."""
    s = tiny_spec(nr=5, nz=8).replace(t_inf=(0.0,) * 4, h=(0.0, 2.0, 2.0, 2.0))
    P = nl_problem(s)
    z = np.zeros((5, 4))
    lam, cap, _ = mild_laws(s, beta=0.1, gamma=0.1)
    P.set_laws(lam, cap, z)
    res = P.nl_run(P.initial(0.0), 0.0, 1.0, kind="erf", pulse_args=(0.02, 0.005, 1e-4, 4.0, 2.0),
                   eps=1e-10, iter_max=20, periodic_tol=1e-9)
    assert res["periodic"] and abs(res["t"] - 0.02) < 1e-15
    lam, cap, src = mild_laws(s, beta=0.1, gamma=0.1, chi=0.1)
    P.set_laws(lam, cap, src)
    args = (0.02, 0.005, 1e-4, 4.0, 2.0)
    res = P.nl_run(P.initial(0.0), 0.0, 50.0, kind="erf", pulse_args=args, eps=1e-10, iter_max=20,
                   periodic_tol=1e-4, tau_trs_div=10.0)
    assert res["periodic"]
    k = round(res["t"] / args[0])
    assert abs(res["t"] - k * args[0]) < 1e-12 and k >= 2
    more = P.nl_run(res["T"], res["t"], res["t"] + args[0], kind="erf", pulse_args=args, eps=1e-10,
                    iter_max=20, tau_trs_div=10.0)
    assert np.max(np.abs(more["T"] - res["T"])) < 1e-4
