"""GPU parity of the HIP ADI solver against the CPU FP64 oracle, element by
element on the same seeded inputs (infinity-norm relative error over active
cells <= 1e-12), plus region maps (bit-exact), profiles, energy and the
launch shapes the autotuner can pick."""
import math

import numpy as np
import pytest

import oracle
from helpers import gpu_available, rel_inf, run_gpu, run_oracle, tiny_spec
from paper_1912_03744_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = 1e-12


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("spec", [tiny_spec(), W.single_layout(), W.production(0, nr=300, nz=700),
                                  W.production(1)],
                         ids=["tiny", "single", "mid", "production"])
def test_region_map_bit_exact(spec):
    from paper_1912_03744_amd import native
    _say("region map %dx%d" % (spec.nr, spec.nz))
    p = native.Problem.from_spec(spec)
    assert np.array_equal(p.region_map(), oracle.Problem.from_spec(spec).region_map())


@pytest.mark.parametrize("scheme", ["pr", "lod"])
@pytest.mark.parametrize("nr,nz", [(7, 12), (5, 9), (13, 31)])
def test_tiny_all_boundary_classes(scheme, nr, nz):
    s = tiny_spec(nr=nr, nz=nz, scheme=scheme)
    _say("tiny %s %dx%d" % (scheme, nr, nz))
    P, want, _ = run_oracle(s, 7)
    p, got = run_gpu(s, 7)
    act = P.active()
    assert np.all(np.isnan(got[~act]))
    assert rel_inf(got, want, act) <= TOL


@pytest.mark.parametrize("scheme", ["lod", "pr"])
def test_single_layout_full_run(scheme):
    """The fixed 64 x 160 instance, dt = 1e-3, 1000 steps, and its 64-point
    terminal-face profile."""
    s = W.single_layout(scheme=scheme)
    _say("single layout %s" % scheme)
    P, want, _ = run_oracle(s, s.nsteps)
    p, got = run_gpu(s, s.nsteps)
    act = P.active()
    assert rel_inf(got, want, act) <= TOL
    prof = p.profile(0, 64)
    wprof = P.profile(want, 0, 64)
    assert np.max(np.abs(prof - wprof)) <= TOL * np.max(np.abs(wprof))
    prof1 = p.profile(1, 50)
    assert np.max(np.abs(prof1 - P.profile(want, 1, 50))) <= TOL * np.max(np.abs(wprof))


def _shapes():
    from paper_1912_03744_amd import native
    return native.launch_shapes()


@pytest.mark.parametrize("shape", _shapes() if gpu_available() else [],
                         ids=lambda s: "m%d_l%d_w%d_r%d_g%d" % s)
def test_launch_shapes_ragged(shape):
    """Every compiled launch shape on grids whose lines are not multiples of
    any chunking (ragged tails, chunks that are pure padding, line groups cut
    short at class boundaries) in both directions and both schemes."""
    m, lpw, wpl, r, ngw = shape
    G = (64 // lpw) * wpl
    ran = 0
    for nr, nz in ((13, 29), (29, 13), (37, 91), (150, 333), (1030, 2570)):
        s = W.production(3, nr=nr, nz=nz).replace(dt=2e-3)
        for d, n in ((0, s.nr), (1, s.nz)):
            if G * m < n or (G * m > 4 * n and n > 100):
                continue
            for scheme in (("pr", "lod") if nr < 1000 else ("pr",)):
                ss = s.replace(scheme=scheme)
                _say("shape %s grid %dx%d dir %d scheme %s" % (shape, nr, nz, d, scheme))
                steps = 5 if nr < 1000 else 1
                P, want, _ = run_oracle(ss, steps)
                p, got = run_gpu(ss, steps, launch={d: shape})
                assert rel_inf(got, want, P.active()) <= TOL, (shape, d, scheme)
                ran += 1
    if not ran:
        pytest.skip("shape covers none of the line lengths")


def _strip_shapes():
    from paper_1912_03744_amd import native
    return [(d, sh) for d in (0, 1) for sh in native.layout_shapes("strips", d)]


@pytest.mark.parametrize("dshape", _strip_shapes() if gpu_available() else [],
                         ids=lambda x: "d%d_m%d_w%d" % (x[0], x[1][0], x[1][2]))
def test_strip_layout_shapes_ragged(dshape):
    """Every strip-layout kernel (right-hand sides in strips of 4 columns) on
    grids with partial strips and partial row groups, strips and row groups
    straddling class boundaries, both schemes."""
    d, shape = dshape
    m, _, nw, _, _ = shape
    cover = 64 * nw * m
    ran = 0
    for nr, nz in ((37, 91), (150, 333), (1030, 2570), (1024, 2560)):
        n = nr if d == 0 else nz
        if cover < n or (cover > 4 * n and n > 100):
            continue
        s = W.production(3, nr=nr, nz=nz).replace(dt=2e-3)
        for scheme in (("pr", "lod") if nr < 1000 else ("pr",)):
            ss = s.replace(scheme=scheme)
            _say("strip shape %s grid %dx%d dir %d scheme %s" % (shape, nr, nz, d, scheme))
            steps = 5 if nr < 1000 else 2
            P, want, _ = run_oracle(ss, steps)
            p, got = run_gpu(ss, steps, launch={d: shape}, layout="strips")
            assert p.layout() == "strips"
            assert rel_inf(got, want, P.active()) <= TOL, (shape, d, scheme)
            ran += 1
    if not ran:
        pytest.skip("shape covers none of the line lengths")


@pytest.mark.parametrize("nr,nz", [(2048, 3072), (2045, 3069)], ids=["max", "max_ragged"])
def test_strip_layout_maximum_line_lengths(nr, nz):
    """The longest lines the strip kernels take (2048-cell rows, 3072-cell
    columns) and a ragged grid just below them (a partial strip and a
    partial row group), in the default strip shapes, with ambient films and
    a non-zero start: full field against the oracle."""
    s = W.production(2, nr=nr, nz=nz).replace(dt=1e-3, t_inf=(0.0, 0.2, -0.1, 0.05), T0=0.1)
    _say("strip layout at the maximum line lengths: %dx%d" % (nr, nz))
    P, want, _ = run_oracle(s, 2)
    p, got = run_gpu(s, 2, layout="strips")
    assert p.layout() == "strips"
    assert rel_inf(got, want, P.active()) <= TOL


@pytest.mark.parametrize("scheme", ["pr", "lod"])
def test_strip_layout_ambient_films_and_checks(scheme):
    """Strip layout with non-zero ambient temperatures on every face class
    (the crossing constants), a Dirichlet class, a non-uniform start field,
    periodic energy checks and graphs, against the oracle; then a switch back
    to the rows layout continues from the same state."""
    from paper_1912_03744_amd import native
    base = tiny_spec(scheme=scheme, dt=0.02)
    for nr, nz in ((7, 12), (61, 203)):
        s = base.replace(nr=nr, nz=nz)
        P = oracle.Problem.from_spec(s)
        rng = np.random.default_rng(nr)
        T0 = np.where(P.active(), rng.uniform(0.0, 1.0, P.shape), 0.0)
        want, _ = P.step(T0, s.scheme, s.dt, 30)
        want2, _ = P.step(want, s.scheme, s.dt, 10)
        _say("strip ambient %s %dx%d" % (scheme, nr, nz))
        p = native.Problem.from_spec(s)
        p.set_layout("strips")
        p.set_field(T0)
        p.set_graph_steps(10)
        p.set_check(10)
        p.step(s.dt, 30)
        assert rel_inf(p.read_field(), want, P.active()) <= TOL
        p.set_layout("rows")
        p.step(s.dt, 10)
        assert rel_inf(p.read_field(), want2, P.active()) <= TOL


def test_production_full_size_short_run(tmp_path, monkeypatch):
    """1024 x 2560 at the production time step, in the launch shapes the
    autotuner picks for the benchmark (and in the default shapes): full-field
    parity after 4 steps (both schemes)."""
    from paper_1912_03744_amd import autotune
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    for scheme in ("pr", "lod"):
        s = W.production(0, scheme=scheme)
        P, want, _ = run_oracle(s, 4)
        for tune, layout in ((False, None), (False, "strips"), (True, None)):
            _say("production full size %s tuned=%s layout=%s" % (scheme, tune, layout))
            p, got = run_gpu(s, 4, tune=tune, layout=layout)
            assert rel_inf(got, want, P.active()) <= TOL


def test_production_energy_identity_long_run():
    """At full size and full length the per-step energy identity is checked
    on the device every 100 steps; here 2000 steps with checks every 50 and
    a graph of 50 steps, and the final field is finite and non-negative
    (Q >= 0, T0 = T_inf = 0: maximum principle holds for the L-stable
    scheme)."""
    s = W.production(2, scheme="lod")
    _say("production energy lod")
    p, got = run_gpu(s, 2000, graph_steps=50, check_every=50)
    e = p.energy()
    assert e["checks"] == 40
    assert e["residual"] < 1e-11
    assert np.nanmin(got) >= 0.0


def _host_threads():
    import os
    n = os.cpu_count() or 1
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, min(n, 16))


@pytest.mark.timeout(900)
def test_production_benchmark_configuration_full_length(tmp_path, monkeypatch):
    """The benchmark's run itself (seed 0, Peaceman-Rachford, dt = 1e-4,
    10,000 steps, graphs of 100 steps, energy identity checked on the device
    every 100 steps, autotuned layout and shapes) against the oracle over the
    whole run: full-field infinity-norm relative error <= 1e-12 at steps
    100, 1000, 3000 and 10,000 (the oracle's line solves shared among the
    host's threads, bit-identical to its serial path), all 100 device checks
    at rounding level."""
    from paper_1912_03744_amd import autotune
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    s = W.production(0)
    P = oracle.Problem.from_spec(s)
    act = P.active()
    want = P.initial(s.T0)
    from paper_1912_03744_amd import native
    p = native.Problem.from_spec(s)
    autotune.apply(p, s.dt, s.scheme)
    p.set_check(100, 1e-9)
    p.set_graph_steps(100)
    done = 0
    threads = _host_threads()
    for upto in (100, 1000, 3000, 10_000):
        p.step(s.dt, upto - done)
        got = p.read_field()
        want, _ = P.step_threads(want, s.scheme, s.dt, upto - done, threads)
        done = upto
        err = rel_inf(got, want, act)
        _say("production full length: step %d, rel err %.3e (layout %s, r %s, z %s)"
             % (upto, err, p.layout(), p.get_launch(0), p.get_launch(1)))
        assert err <= TOL, (upto, err)
    e = p.energy()
    assert e["checks"] == 100
    assert e["residual"] < 1e-12


@pytest.mark.parametrize("seed", [1, 2])
def test_production_other_seeds(tmp_path, monkeypatch, seed):
    """The production grid with the other seeded material sets (seeds 1 and
    2 of the benchmark's generator), in the benchmark's configuration
    (autotuned layout and shapes, graphs of 100 steps, checks every 100):
    full-field parity with the oracle after 300 steps."""
    from paper_1912_03744_amd import autotune, native
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    s = W.production(seed)
    P = oracle.Problem.from_spec(s)
    want, _ = P.step_threads(P.initial(s.T0), s.scheme, s.dt, 300, _host_threads())
    p = native.Problem.from_spec(s)
    autotune.apply(p, s.dt, s.scheme)
    p.set_check(100, 1e-9)
    p.set_graph_steps(100)
    p.step(s.dt, 300)
    err = rel_inf(p.read_field(), want, P.active())
    _say("production seed %d: 300 steps, rel err %.3e" % (seed, err))
    assert err <= TOL
    assert p.energy()["residual"] < 1e-11


def test_graph_and_checks_do_not_change_results():
    s = W.production(1, nr=200, nz=500)
    _say("graph vs plain")
    _, a = run_gpu(s, 120)
    _, b = run_gpu(s, 120, graph_steps=30, check_every=30)
    _, c = run_gpu(s, 120, graph_steps=40)
    act = ~np.isnan(a)
    assert np.array_equal(a[act], b[act]) and np.array_equal(a[act], c[act])


def test_energy_report_matches_oracle():
    s = tiny_spec(nr=11, nz=17)
    P, want, _ = run_oracle(s, 9)
    p, got = run_gpu(s, 9)
    e = p.energy()
    o = P.energy(want)
    assert abs(e["E"] - o["E"]) <= 1e-12 * abs(o["E"])
    assert abs(e["source_power"] - o["P"]) <= 1e-13 * abs(o["P"])
    assert abs(e["boundary_flow"] - (o["Br"] + o["Bz"])) <= 1e-11 * (abs(o["Br"]) + abs(o["Bz"]))
    assert e["steps"] == 9 and abs(e["time"] - 9 * s.dt) < 1e-15


def test_nonuniform_layer_aligned_grid():
    """Face arrays uniform inside each layer (the grid style of Sec. 5),
    with strongly different cell widths."""
    r_f = W.layer_aligned_faces((0.0, 2.0, 3.0, 4.0, 4.2), (20, 7, 9, 3))
    z_f = W.layer_aligned_faces((0.0, 8.0, 10.0, 10.2), (30, 12, 4))
    s = W.single_layout(nr=39, nz=46, scheme="pr").replace(r_faces=r_f, z_faces=z_f, dt=5e-3)
    P, want, _ = run_oracle(s, 40)
    p, got = run_gpu(s, 40)
    assert rel_inf(got, want, P.active()) <= TOL
    assert np.array_equal(p.region_map(), P.region_map())


@pytest.mark.parametrize("scheme", ["lod", "pr"])
def test_case_study_grid_linear(scheme):
    """The case-study grid of Sec. 5 through the face arrays (per-layer
    uniform faces, 800/200/200/10 x 80/20 cells, widths down to 1e-5 against
    0.05 in z), T0 held on the top face (Dirichlet, eq. 6), insulated
    elsewhere, constant coefficients with a heater source: 200 steps of 1e-4.
    The coating cells couple about 1e6 times more strongly than their
    capacity term (tau k / (dr^2 rho c)), so both schemes are held to the
    rounding bound stiff_tol (see test_nonlinear_emulation.py) instead of
    1e-12: two correct line solvers differ by about eps times that ratio
    per solve, Peaceman-Rachford's explicit half adds the same amount, and
    with weights tau / 2 (PR) or tau (LOD backward Euler) per half step the
    bound is 4 eps sum(weight * max coupling ratio).  Measured: about 1e-11
    against bounds near 1e-7."""
    from test_nonlinear_emulation import stiff_tol
    s = W.case_study().replace(scheme=scheme)
    _say("case-study grid %dx%d linear %s" % (s.nr, s.nz, scheme))
    P, want, _ = run_oracle(s, 200)
    p, got = run_gpu(s, 200)
    tol = stiff_tol(P, [s.dt if scheme == "pr" else 2 * s.dt] * 200, 1.0)
    err = rel_inf(got, want, P.active())
    _say("case-study grid %s: rel err %.2e (bound %.2e)" % (scheme, err, tol))
    assert err <= tol
    assert np.max(np.abs(want[P.active()] - s.T0)) > 1e-6  # the heater has warmed the cell


def test_set_field_and_continuation():
    """Stepping 3 + 4 equals stepping 7; a host field is accepted; changing
    dt rebuilds the tables."""
    s = tiny_spec(nr=20, nz=33)
    rng = np.random.default_rng(0)
    P = oracle.Problem.from_spec(s)
    T0 = np.where(P.active(), rng.uniform(0, 1, P.shape), 0.0)
    want, _ = P.step(T0, s.scheme, s.dt, 7)
    want, _ = P.step(want, s.scheme, 2 * s.dt, 2)
    from paper_1912_03744_amd import native
    p = native.Problem.from_spec(s)
    p.set_field(T0)
    p.step(s.dt, 3)
    p.step(s.dt, 4)
    p.step(2 * s.dt, 2)
    assert rel_inf(p.read_field(), want, P.active()) <= TOL


def test_state_errors():
    from paper_1912_03744_amd import native
    s = tiny_spec()
    p = native.Problem(s.geom, s.nr, s.nz, s.h, s.t_inf)
    with pytest.raises(native.AdiError) as e:
        p.step(0.1, 1)
    assert e.value.status == native.ADI_ESTATE
    p.set_materials(s.k, s.rhoc)
    with pytest.raises(native.AdiError):
        p.set_materials((1, 1, -1, 1, 1), s.rhoc)
    with pytest.raises(native.AdiError) as e:
        p.set_sources((0, 0, math.nan, 0, 0))
    assert e.value.status == native.ADI_ENONFINITE
    p.set_sources(s.q)
    with pytest.raises(native.AdiError):
        p.step(-1.0, 1)
    p.step(0.1, 1)
    with pytest.raises(native.AdiError):
        p.set_launch(0, 2, 4, 1, 1, 1)
