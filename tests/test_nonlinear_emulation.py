"""The nonlinear path's persistent kernel (paper_1912_03744_amd/csrc/
nonlinear.hpp: the simple iteration of eq. 12 and eq. 14 with the stop rule
of eq. 13, step halving, the pulsed source of eq. 2-4 and the step rule of
Sec. 4) compiled for the host with the stand-in for the HIP device
environment (tests/emu/shim), every workgroup on a host thread as in the
cooperative launch, against the oracle's nonlinear path: one attempt (field,
solves of each half, accepted or not), adaptive runs through transitions of
the pulse (every step's time, size and solves, the final field), forced
halving, the periodic stop, grids with fewer workgroups than lines, layer-
aligned non-uniform faces with a Dirichlet top face.

The stop decisions compare a change norm with eps; both sides take them in
FP64 on fields that differ by rounding only, so every case checks that its
decisions were far from a tie (the oracle's smallest margin) before it
requires equal counts."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from helpers import rel_inf
from paper_1912_03744_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = 1e-12
PULSE = (0.1, 0.01, 1e-4, 4.0, 2.0)   # t_per, t_src, t_trs, xi, zeta (Sec. 5, Fig. 2)
KINDS = {"const": 0, "rect": 1, "erf": 2}

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    exe = tmp_path_factory.mktemp("nlemu") / "nl_emu"
    cmd = ["g++", "-std=c++20", "-O1", "-Wno-unknown-pragmas", "-Wno-attributes",
           "-I", os.path.join(ROOT, "tests", "emu", "shim"),
           "-I", os.path.join(ROOT, "paper_1912_03744_amd", "csrc"),
           os.path.join(ROOT, "tests", "emu", "nl_emu.cpp"), "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True)
    return exe


def tiny_spec(nr=7, nz=12):
    """Every region, the cut-out, the terminal and all four face classes,
    non-zero ambient temperatures and one Dirichlet class."""
    return W.Spec(r0=1.0, r1=1.6, r2=2.3, rmax=2.6, z0=3.1, zmax=4.4, ztop=5.0, nr=nr, nz=nz,
                  h=(0.3, 0.2, math.inf, 0.15), t_inf=(0.4, -0.3, 0.25, 0.1),
                  k=(0.8, 0.07, 1.3, 0.2, 2.1), rhoc=(1.1, 0.6, 1.7, 0.9, 1.3),
                  q=(0.2, 0.0, 1.5, 0.3, 0.1))


def laws_of(s, beta=0.3, gamma=0.2, chi=0.1):
    lam = np.zeros((5, 4))
    cap = np.zeros((5, 4))
    src = np.zeros((5, 4))
    lam[:, 0], lam[:, 1] = s.k, np.asarray(s.k) * beta
    cap[:, 0], cap[:, 2] = s.rhoc, np.asarray(s.rhoc) * gamma
    src[:, 0], src[:, 1] = s.q, np.asarray(s.q) * chi
    return lam, cap, src


def nl_problem(s, laws):
    P = oracle.NonlinearProblem(s.geom, s.nr, s.nz, s.h, s.t_inf, s.k, s.rhoc, s.q, s.r_faces, s.z_faces)
    P.set_laws(*laws)
    return P


def run_emu(emu, tmp_path, s, laws, T, *, grid, mode, kind="const", pulse=PULSE, eps=1e-10, iter_max=10,
            tau_min=1e-14, div_trs=1000.0, div_src=100.0, ptol=0.0, t0=0.0, t_end_or_tau=1e-3,
            max_steps=1 << 40, log_cap=0, z_block=False, polls=None):
    """z_block: solve the z lines with a whole workgroup each (the long-line
    path) instead of one wave each; polls: bound of every grid-wide wait
    (ADI_NL_WAIT_POLLS), None for the library's default."""
    inp, out = tmp_path / "in.txt", tmp_path / "out.txt"
    fmt = lambda v: " ".join("%.17g" % x for x in np.ravel(v))
    faces = s.r_faces is not None
    lines = ["%d %d %d %d" % (s.nr, s.nz, grid, mode), fmt(s.geom), "1" if faces else "0"]
    if faces:
        lines += [fmt(s.r_faces), fmt(s.z_faces)]
    lines += [fmt(s.h).replace("inf", "inf"), fmt(s.t_inf), fmt(laws[0]), fmt(laws[1]), fmt(laws[2]),
              "%d %s" % (KINDS[kind], fmt(pulse)), "%.17g %d %.17g %.17g %.17g %.17g" % (
                  eps, iter_max, tau_min, div_trs, div_src, ptol),
              "%.17g %.17g %d %d" % (t0, t_end_or_tau, min(max_steps, 1 << 60), log_cap), fmt(T)]
    inp.write_text("\n".join(lines) + "\n")
    env = dict(os.environ)
    if z_block:
        env["NL_EMU_WZ_BLOCK"] = "1"
    env.pop("ADI_NL_WAIT_POLLS", None)
    if polls is not None:
        env["ADI_NL_WAIT_POLLS"] = str(polls)
    subprocess.run([str(emu), str(inp), str(out)], check=True, timeout=600, env=env)
    rows = out.read_text().split("\n")
    h = rows[0].split()
    res = {"status": int(h[0]), "t": float(h[1]), "steps": int(h[2]), "rejected": int(h[3]),
           "solves_r": int(h[4]), "solves_z": int(h[5]), "min_margin": float(h[6]),
           "it": (int(h[7]), int(h[8])), "chg": (float(h[9]), float(h[10])), "accepted": bool(int(h[11]))}
    nlog = min(res["steps"], log_cap)
    res["log"] = np.array([[float(x) for x in r.split()] for r in rows[1:1 + nlog]]).reshape(-1, 4)
    res["T"] = np.array([float(x) for x in rows[1 + nlog:1 + nlog + s.nr * s.nz]]).reshape(s.nz, s.nr)
    return res


@pytest.mark.parametrize("z_block", [False, True], ids=["z_wave", "z_block"])
def test_single_attempt_matches_oracle(emu, tmp_path, z_block):
    """One attempt at a fixed tau on a tiny grid with every face class: the
    solves of each half step equal the oracle's, the field agrees to 1e-12;
    z lines on one wave each and on a whole workgroup each."""
    s = tiny_spec(13, 31)
    laws = laws_of(s)
    P = nl_problem(s, laws)
    T0 = P.initial(0.5)
    for tau in (0.02, 0.08):
        ok, want, its, chg = P.nl_step(T0, tau, 0.0, eps=1e-10, iter_max=30)
        assert ok and min(its) >= 3
        assert min(abs(c - 1e-10) / 1e-10 for c in chg) > 1e-3
        got = run_emu(emu, tmp_path, s, laws, T0, grid=7, mode=1, eps=1e-10, iter_max=30, t_end_or_tau=tau,
                      z_block=z_block)
        assert got["status"] == 4 and got["accepted"]
        assert got["it"] == its
        assert rel_inf(got["T"], want, P.active()) <= TOL


def test_constant_laws_one_solve_equals_linear_step(emu, tmp_path):
    """With laws equal to the linear problem's constants the iteration stops
    after its second solve (the first changes T, the second reproduces it)
    and one step equals the linear Peaceman-Rachford step of the oracle."""
    s = tiny_spec(11, 23)
    z = np.zeros((5, 3))
    laws = (np.column_stack([s.k, z]), np.column_stack([s.rhoc, z]), np.column_stack([s.q, z]))
    P = oracle.Problem.from_spec(s)
    T0 = P.initial(0.3)
    want, _ = P.step(T0, "pr", 0.1, 1)
    got = run_emu(emu, tmp_path, s, laws, T0, grid=5, mode=1, eps=1e-9, t_end_or_tau=0.1)
    assert got["accepted"] and got["it"] == (2, 2)
    assert rel_inf(got["T"], want, P.active()) <= TOL


def test_iteration_limit_rejects_attempt(emu, tmp_path):
    """An attempt whose iteration cannot stop within iter_max solves is
    rejected and leaves the field unchanged (single-attempt mode)."""
    s = tiny_spec(9, 17)
    laws = laws_of(s, beta=2.0, gamma=1.0, chi=1.0)
    P = nl_problem(s, laws)
    T0 = P.initial(0.5)
    ok, _, its, _ = P.nl_step(T0, 0.5, 0.0, eps=1e-12, iter_max=2)
    assert not ok and its[0] == -1
    got = run_emu(emu, tmp_path, s, laws, T0, grid=4, mode=1, eps=1e-12, iter_max=2, t_end_or_tau=0.5)
    assert not got["accepted"] and got["it"] == its
    act = P.active()
    assert np.array_equal(got["T"][act], T0[act])


@pytest.mark.parametrize("kind", ["rect", "erf"])
def test_adaptive_run_through_transitions(emu, tmp_path, kind):
    """The time loop over the first switch-on transition, the heating and
    the switch-off: every accepted step's start time, size and solves equal
    the oracle's, and the final field agrees to 1e-12."""
    s = tiny_spec(10, 21)
    laws = laws_of(s)
    P = nl_problem(s, laws)
    T0 = P.initial(0.2)
    pulse = (0.02, 0.004, 2e-4, 4.0, 2.0)
    kw = dict(kind=kind, pulse_args=pulse, eps=1e-10, iter_max=12, tau_trs_div=20.0, tau_src_div=10.0)
    want = P.nl_run(T0, 0.0, 0.0062, log_cap=4000, **kw)
    assert want["steps"] > 30 and want["min_margin"] > 1e-3
    got = run_emu(emu, tmp_path, s, laws, T0, grid=6, mode=0, kind=kind, pulse=pulse, eps=1e-10, iter_max=12,
                  div_trs=20.0, div_src=10.0, t_end_or_tau=0.0062, log_cap=4000)
    assert got["status"] == 1
    for key in ("steps", "rejected", "solves_r", "solves_z"):
        assert got[key] == want[key], key
    assert np.array_equal(got["log"][:, 2:], want["log"][:, 2:])
    assert np.allclose(got["log"][:, :2], want["log"][:, :2], rtol=0, atol=1e-15)
    assert abs(got["t"] - want["t"]) <= 1e-15
    assert rel_inf(got["T"], want["T"], P.active()) <= TOL


def test_wait_bound_aborts_the_run(emu, tmp_path):
    """A grid-wide wait that runs out of polls aborts the run: the waiting
    wave raises the abort flag, every other wave leaves at its next wait,
    the kernel returns and the run reports the failed wait (status -2)
    instead of hanging.  With one workgroup no wait ever polls, so the same
    bound lets the run finish."""
    s = tiny_spec(8, 15)
    laws = laws_of(s)
    P = nl_problem(s, laws)
    T0 = P.initial(0.3)
    kw = dict(kind="const", eps=1e-10, t_end_or_tau=0.01)
    got = run_emu(emu, tmp_path, s, laws, T0, grid=4, mode=0, polls=0, **kw)
    assert got["status"] == -2
    one = run_emu(emu, tmp_path, s, laws, T0, grid=1, mode=0, polls=0, **kw)
    want = P.nl_run(T0, 0.0, 0.01, kind="const", eps=1e-10)
    assert one["status"] == 1 and one["steps"] == want["steps"]
    assert rel_inf(one["T"], want["T"], P.active()) <= TOL


def test_forced_halving_matches_oracle(emu, tmp_path):
    """An iteration limit of 2 with strongly T-dependent laws: attempts fail
    and are retried with half the step; the number of rejections and every
    accepted step agree with the oracle."""
    s = tiny_spec(8, 15)
    laws = laws_of(s, beta=1.5, gamma=0.8, chi=0.5)
    P = nl_problem(s, laws)
    T0 = P.initial(0.4)
    kw = dict(kind="const", eps=1e-6, iter_max=3, tau_src_div=1.0)
    want = P.nl_run(T0, 0.0, 0.05, pulse_args=(0.1, 0.2, 1e-4, 4.0, 2.0), log_cap=1000, **kw)
    assert want["rejected"] > 0 and want["min_margin"] > 1e-3
    got = run_emu(emu, tmp_path, s, laws, T0, grid=3, mode=0, kind="const", pulse=(0.1, 0.2, 1e-4, 4.0, 2.0),
                  eps=1e-6, iter_max=3, div_src=1.0, t_end_or_tau=0.05, log_cap=1000)
    for key in ("steps", "rejected", "solves_r", "solves_z"):
        assert got[key] == want[key], key
    assert np.allclose(got["log"], want["log"], rtol=0, atol=1e-15)
    assert rel_inf(got["T"], want["T"], P.active()) <= TOL


def test_periodic_stop_matches_oracle(emu, tmp_path):
    """The periodic-regime stop: the run ends at the same period start as the
    oracle's, with the same field."""
    s = tiny_spec(6, 11)
    laws = laws_of(s, beta=0.1, gamma=0.1, chi=0.05)
    P = nl_problem(s, laws)
    T0 = P.initial(0.0)
    pulse = (0.5, 0.1, 0.01, 4.0, 2.0)
    kw = dict(kind="erf", pulse_args=pulse, eps=1e-10, iter_max=12, tau_trs_div=4.0, tau_src_div=5.0)
    want = P.nl_run(T0, 0.0, 400.0, periodic_tol=2e-3, **kw)
    assert want["periodic"] and want["min_margin"] > 1e-3
    got = run_emu(emu, tmp_path, s, laws, T0, grid=4, mode=0, kind="erf", pulse=pulse, eps=1e-10, iter_max=12,
                  div_trs=4.0, div_src=5.0, ptol=2e-3, t_end_or_tau=400.0)
    assert got["status"] == 2
    assert got["steps"] == want["steps"] and got["rejected"] == want["rejected"]
    assert abs(got["t"] - want["t"]) <= 1e-12
    assert rel_inf(got["T"], want["T"], P.active()) <= TOL


def stiff_tol(P, taus, law_factor):
    """Rounding bound of a Peaceman-Rachford run with stiff explicit halves.
    Each half step applies one direction's operator explicitly and solves the
    other; with D = tau/2 max |diagonal / rho c| (the largest explicit
    coupling of a cell), both the explicit sum and the solve lose up to about
    eps D relative to T, and PR does not damp the stiffest modes (their
    amplification tends to -1), so the difference between two correct
    implementations can grow like the sum of D over the steps.  Bound:
    4 eps sum_steps D, never below 1e-12; law_factor bounds lambda / rho c_V
    of the laws against the constants over the temperatures reached."""
    act = P.active()
    C = P.coeffs("C")[act]
    D = max(np.abs(P.coeffs("Lr_c")[act] / C).max(), np.abs(P.coeffs("Lz_c")[act] / C).max()) * law_factor
    return max(TOL, 4 * np.finfo(float).eps * float(np.sum(0.5 * np.asarray(taus) * D)))


def test_layer_aligned_faces_dirichlet_top(emu, tmp_path):
    """The case-study layout of Sec. 5 in miniature: per-layer uniform faces
    (core, two thin layers, a thinner coating: widths 3e-2 down to 5e-5
    against 0.5 in z), no terminal slab, T0 held on the top face (Dirichlet,
    eq. 6), insulated elsewhere.  The explicit r half is stiff here (tau/2
    times the coating's coupling reaches 2e4), so the field is held to the
    rounding bound of stiff_tol (about 6e-11 here) rather than 1e-12; the
    step sequence must still agree exactly."""
    rf = np.concatenate([np.linspace(0, 0.24, 9), np.linspace(0.24, 0.245, 4)[1:], np.linspace(0.245, 0.25, 4)[1:],
                         np.linspace(0.25, 0.2501, 3)[1:]])
    zf = np.concatenate([np.linspace(0, 4.0, 9), np.linspace(4.0, 5.0, 4)[1:]])
    s = W.Spec(r0=0.24, r1=0.245, r2=0.25, rmax=0.2501, z0=4.0, zmax=5.0, ztop=5.0, nr=len(rf) - 1,
               nz=len(zf) - 1, h=(0.0, 0.0, math.inf, 0.0), t_inf=(0.0, 0.0, 4.2, 0.0),
               k=(40.0, 0.5, 2.0, 1.0, 1.0), rhoc=(1.0, 1.5, 1.2, 1.1, 1.0), q=(0.0, 0.0, 300.0, 0.0, 0.0),
               r_faces=rf, z_faces=zf)
    laws = laws_of(s, beta=0.02, gamma=0.01, chi=0.01)
    P = nl_problem(s, laws)
    T0 = P.initial(4.2)
    pulse = (0.1, 0.01, 1e-4, 4.0, 2.0)
    kw = dict(kind="erf", pulse_args=pulse, eps=1e-9, iter_max=15)
    want = P.nl_run(T0, 0.0, 0.0003, log_cap=2000, **kw)
    assert want["min_margin"] > 1e-3
    got = run_emu(emu, tmp_path, s, laws, T0, grid=5, mode=0, kind="erf", pulse=pulse, eps=1e-9, iter_max=15,
                  t_end_or_tau=0.0003, log_cap=2000)
    for key in ("steps", "rejected", "solves_r", "solves_z"):
        assert got[key] == want[key], key
    lin = oracle.Problem.from_spec(s)
    # lambda grows by 2 % per unit of T and rho c_V by 1 % per unit of T^2:
    # at T <= 6 the ratio stays below 1.12 times the constants'
    assert np.abs(want["T"][P.active()]).max() < 6.0
    tol = stiff_tol(lin, want["log"][:, 1], 1.12)
    assert tol < 1e-9
    assert rel_inf(got["T"], want["T"], P.active()) <= tol
