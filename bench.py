"""Benchmark: ADI time stepping of the production-resolution problem on one
MI355X.

Workload: the layered-cylinder layout at 1024 (r) x 2560 (z) cells, seeded
materials (seed 0), Peaceman-Rachford steps of dt = 1e-4 with the device
energy-identity check every 100 steps.  A step is one full ADI step: the
r-implicit sweep and the z-implicit sweep over the whole grid (and, every 100
steps, the three energy reductions and the identity check).

Prints one JSON line:
  value       active-cell updates per second (cells inside the domain x steps
              / wall time, inputs resident in HBM)
  roofline    the dominant sweep kernel against MI355X's 8 TB/s HBM peak:
              algorithmic bytes per launch (16 B per active cell: the
              right-hand side read once and the next one written once) over
              its mean launch time, measured with HIP events on the stream
              the kernel runs on
  cpu_baseline  the CPU FP64 oracle timed on a bounded sample of the same
              workload on this host's cores (its line solves shared among
              OpenMP threads, as in the paper; single-threaded figure beside)
  single_layout  secondary figure: the 64x160 layout of Fig. 1, 1000 steps
              (latency-bound; microseconds per step)
  surrogate_training  secondary figure: Adam steps of the surrogate's network
              (batch 4096), samples/s and the matrix-core fraction
  batch       secondary figure: the ragged design batch (4096 seeded
              instances of 64x160 ... 192x480 cells, 2000 PR steps of 1e-3)
              as captured graphs: a persistent kernel or batched sweep
              launches, whichever the autotuner picks; cell-updates/s and the
              algorithmic bandwidth (32 B per active cell per step)
Usage: python bench.py [--gpus 1] [--steps 10000] [--warmup 200] [--no-batch]
       python bench.py --counter-workload [batch]        (the program profiled for traffic)
       python bench.py --summarize-counters DIR [batch]  (rocprofv3 --pmc output -> profiles/)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_HALF_STEP = 16


# The sources the production sweeps are built and launched from: the counter
# readings stay valid while these are unchanged.
SWEEP_SOURCES = ("common.hpp", "device.hpp", "strip.hpp", "solver.hip")
# ... and those of the batch's batched sweep launches.
BATCH_SOURCES = ("common.hpp", "device.hpp", "strip.hpp", "batch.hpp", "batch.hip")


def source_digest(files=SWEEP_SOURCES):
    """Hash of HIP sources (by default those of the production sweeps), to
    tie stored counter readings to a build."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1912_03744_amd", "csrc")
    for f in files:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def _stored(path, files):
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    return rec if rec.get("source_digest") == source_digest(files) else None


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current sources; else None."""
    rec = _stored(COUNTERS_JSON, SWEEP_SOURCES)
    k = None if rec is None else rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def stored_batch_traffic():
    """HBM bytes per step of the batch's batched sweep launches (every r and
    z launch of one step) from the committed counter summary, if it was taken
    on the current sources; else None."""
    rec = _stored(BATCH_COUNTERS_JSON, BATCH_SOURCES)
    return None if rec is None else rec.get("hbm_bytes_per_step")


def host_threads():
    """Threads for the CPU baseline: the host's share (OMP_NUM_THREADS when
    set), at most the cores the process sees."""
    n = os.cpu_count() or 1
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, n)


def cpu_baseline(spec, steps, threaded_steps):
    """The oracle on a bounded sample of the workload: PR steps of the same
    grid from T0, single-threaded and with the line solves of each half step
    shared among the host's threads (the paper's OpenMP parallelisation; the
    same result bit for bit).  The threaded figure is the baseline."""
    import numpy as np

    import oracle
    P = oracle.Problem.from_spec(spec)
    T = P.initial(spec.T0)
    active = int(np.count_nonzero(P.active()))
    t0 = time.perf_counter()
    P.step(T, spec.scheme, spec.dt, steps)
    dt1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, used = P.step_threads(T, spec.scheme, spec.dt, threaded_steps, host_threads())
    dtn = time.perf_counter() - t0
    return {"value": active * threaded_steps / dtn, "unit": "cell-updates/s", "cores": used, "kind": "oracle",
            "sample": "%d PR steps of the %dx%d grid from T0, C -O2, line solves of each half step on %d "
                      "OpenMP threads" % (threaded_steps, spec.nr, spec.nz, used),
            "seconds": round(dtn, 3),
            "single_thread": {"value": active * steps / dt1, "cores": 1, "steps": steps,
                              "seconds": round(dt1, 3)}}


def batch_cpu_baseline(steps):
    """The oracle on 16 instances of the design batch (4 per size class, the
    batch's own generator), each stepped alone with the host's threads over
    the lines of a half step; extrapolated per cell-update."""
    import numpy as np

    import oracle
    from paper_1912_03744_amd import workloads as W
    specs = W.ragged_batch(64, master_seed=0, scheme="pr", dt=1e-3, nsteps=steps)
    picked, per = [], {}
    for s in specs:
        if per.get((s.nr, s.nz), 0) < 4:
            per[(s.nr, s.nz)] = per.get((s.nr, s.nz), 0) + 1
            picked.append(s)
    updates, sec, used = 0, 0.0, 1
    for s in picked:
        P = oracle.Problem.from_spec(s)
        T = P.initial(s.T0)
        t0 = time.perf_counter()
        _, used = P.step_threads(T, s.scheme, s.dt, steps, host_threads())
        sec += time.perf_counter() - t0
        updates += int(np.count_nonzero(P.active())) * steps
    return {"value": updates / sec, "unit": "cell-updates/s", "cores": used, "kind": "oracle",
            "sample": "%d instances of the batch (%s), %d PR steps each, %d OpenMP threads over the lines "
                      "of each half step; extrapolated per cell-update"
                      % (len(picked), ", ".join("%d of %dx%d" % (c, a, b) for (a, b), c in sorted(per.items())),
                         steps, used),
            "seconds": round(sec, 3)}


def batch_leg(n, steps, tune=True, shape=(2, 8, 1)):
    """The ragged design batch: one timed adi_batch_step call over all
    instances from their initial fields (events on the batch's stream)."""
    from paper_1912_03744_amd import autotune, native
    from paper_1912_03744_amd import workloads as W
    specs = W.ragged_batch(n, master_seed=0, scheme="pr", dt=1e-3, nsteps=steps)
    dt = specs[0].dt
    b = native.Batch(specs, scheme="pr")
    if tune:
        t0 = time.perf_counter()
        tuned = autotune.apply_batch(b, dt, "pr")
        shape, zshape = tuple(tuned["shape"]), list(tuned["zshape"])
        print("bench: batch autotune %.1f s -> %s, z shapes %s" % (time.perf_counter() - t0, tuned["shape"],
                                                                    zshape), file=sys.stderr, flush=True)
    else:
        zshape = [0, 0, 0, 0]
        b.set_launch(*shape)
    mode = ("batched sweep launches (one per half step and line shape), captured 256 steps per graph"
            if shape[1] == 1 else "one persistent launch")
    b.time(dt, 20, 1)  # warm-up (allocates the workgroup scratch)
    ms = b.time(dt, steps, 1)
    active, cells = b.active_cells(), b.cells()
    sec = ms * 1e-3
    achieved = 2 * BYTES_PER_CELL_HALF_STEP * active * steps / sec / 1e9
    info = b.info()
    out = {"workload": "ragged design batch: %d instances, sizes U{64x160, 96x240, 128x320, 192x480}, "
                       "master seed 0, Peaceman-Rachford, dt=%g, %d steps, %s" % (n, dt, steps, mode),
           "value": active * steps / sec, "unit": "cell-updates/s", "cups_all_cells": cells * steps / sec,
           "seconds": sec, "designs_per_s": n / sec, "active_cells": active, "cells": cells,
           "launch": list(shape), "workgroups": info["workgroups"],
           "zshape": {"variant_per_class": zshape,
                      "shapes": [list(native.batch_zshapes()[c]["shapes"][v]) for c, v in enumerate(zshape)]},
           "roofline": {"bound": "hbm", "kernel": "batch", "achieved": achieved, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "traffic": stored_batch_traffic() if shape == (4, 1, 1) and zshape == [0, 0, 0, 0] else None,
                        "traffic_unit": "HBM bytes per step (every r and z launch of one step)",
                        "alg_bytes_per_step": 2 * BYTES_PER_CELL_HALF_STEP * active}}
    b.close()
    return out


COUNTER_COPY_BYTES = 64 << 20
COUNTERS_JSON = os.path.join(ROOT, "profiles", "sweep_counters_production_1024x2560.json")
BATCH_COUNTERS_JSON = os.path.join(ROOT, "profiles", "batch_counters_ragged_4096.json")
BATCH_COUNTER_STEPS = 10


def counter_workload(seed, batch=False):
    """The program profiled for HBM traffic (one rocprofv3 --pmc pass per
    counter): a plain copy of COUNTER_COPY_BYTES (torch.neg, read once and
    written once) to calibrate the counters, then 20 launches of each sweep
    of the production grid in the benchmark's layout and shapes, or (batch)
    BATCH_COUNTER_STEPS steps of the benchmark's 4096-design batch as
    batched sweep launches in the default z shapes."""
    import torch

    from paper_1912_03744_amd import autotune, native
    from paper_1912_03744_amd import workloads as W
    torch.cuda.set_device(0)
    src = torch.ones(COUNTER_COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    if batch:
        specs = W.ragged_batch(4096, master_seed=seed, scheme="pr", dt=1e-3, nsteps=BATCH_COUNTER_STEPS)
        b = native.Batch(specs, scheme="pr")
        b.set_launch(4, 1, 1)
        b.step(specs[0].dt, BATCH_COUNTER_STEPS)
        b.sync()
        print("counter workload done: batch of %d, %d steps" % (len(specs), BATCH_COUNTER_STEPS), flush=True)
        b.close()
        return
    spec = W.production(seed)
    p = native.Problem.from_spec(spec)
    autotune.apply(p, spec.dt, spec.scheme)
    p.step(spec.dt, 2)
    p.time_sweeps(spec.dt, 20)
    print("counter workload done: layout %s r %s z %s" % (p.layout(), p.get_launch(0), p.get_launch(1)), flush=True)


def summarize_counters(root, batch=False):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the sweeps from two
    rocprofv3 --pmc runs of counter_workload (root/fetch, root/write), scaled
    by what the same counters read for the calibration copy, into
    COUNTERS_JSON; or (batch) those of each batched-sweep kernel and their
    sum over one step, into BATCH_COUNTERS_JSON."""
    import csv
    import glob
    import re

    def name_of(k):
        if "neg" in k:
            return "copy"
        if batch:
            # demangled (k_bsweep_z<4, 2>) or mangled (k_bsweep_zILi4ELi2E) names
            m = (re.search(r"k_bsweep_([rz])<(\d+)(?:,\s*(\d+))?>", k) or
                 re.search(r"k_bsweep_([rz])ILi(\d+)E(?:Li(\d+)E)?", k))
            return None if m is None else "batch_%s<%s>" % (m.group(1), ",".join(g for g in m.groups()[1:] if g))
        if re.search(r"k_sweep_rs", k):
            return "sweep_r"
        if re.search(r"k_sweep_zs|k_sweepILi", k):
            return "sweep_z" if "zs" in k else "sweep_rows"
        return None

    def means(pattern):
        out = {}
        files = glob.glob(os.path.join(root, pattern, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit("no counter_collection.csv under %s" % os.path.join(root, pattern))
        for f in files:
            for row in csv.DictReader(open(f)):
                name = name_of(row["Kernel_Name"])
                if name is not None:
                    out.setdefault(name, []).append(float(row["Counter_Value"]))
        return {k: (sum(v) / len(v), len(v)) for k, v in out.items()}
    fetch, write = means("fetch"), means("write")
    f_scale = COUNTER_COPY_BYTES / (fetch["copy"][0] * 1024.0)
    w_scale = COUNTER_COPY_BYTES / (write["copy"][0] * 1024.0)
    rec = {"source_digest": source_digest(BATCH_SOURCES if batch else SWEEP_SOURCES),
           "calibration": {"copy_bytes": COUNTER_COPY_BYTES, "copy_fetch_kib": fetch["copy"][0],
                           "copy_write_kib": write["copy"][0], "fetch_scale": f_scale, "write_scale": w_scale},
           "kernels": {}}
    names = sorted(k for k in fetch if k != "copy") if batch else ("sweep_r", "sweep_z")
    for k in names:
        if k in fetch and k in write:
            fb = fetch[k][0] * 1024.0 * f_scale
            wb = write[k][0] * 1024.0 * w_scale
            rec["kernels"][k] = {"fetch_kib": fetch[k][0], "write_kib": write[k][0], "fetch_bytes": fb,
                                 "write_bytes": wb, "hbm_bytes_per_launch": fb + wb, "dispatches": fetch[k][1]}
    if batch:
        # every batched-sweep kernel runs once per step
        rec["steps"] = BATCH_COUNTER_STEPS
        rec["hbm_bytes_per_step"] = sum(v["hbm_bytes_per_launch"] for v in rec["kernels"].values())
    with open(BATCH_COUNTERS_JSON if batch else COUNTERS_JSON, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def single_layout_leg():
    """The single layout of Fig. 1 at 64 x 160 (latency-bound: the field is
    80 KB): 1000 backward-Euler LOD steps of 1e-3 in one timed call, in the
    autotuned layout and shapes."""
    import numpy as np
    import torch

    from paper_1912_03744_amd import autotune, native
    from paper_1912_03744_amd import workloads as W
    spec = W.single_layout()
    p = native.Problem.from_spec(spec)
    autotune.apply(p, spec.dt, spec.scheme)
    p.set_graph_steps(100)
    p.step(spec.dt, 100)
    p.read_field()
    p.set_field(None, spec.T0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.step(spec.dt, spec.nsteps)
    T = p.read_field()
    wall = time.perf_counter() - t0
    active = int(np.count_nonzero(~np.isnan(T)))
    out = {"workload": "single layout of Fig. 1, 64x160, LOD backward Euler, dt=1e-3, 1000 steps",
           "value": active * spec.nsteps / wall, "unit": "cell-updates/s", "us_per_step": wall * 1e6 / spec.nsteps,
           "active_cells": active, "layout": p.layout(), "terminal_peak": float(np.nanmax(T[-1]))}
    p.close()
    return out


def mlp_flop_per_sample(widths):
    """Products of one forward pass: 2 * sum of n_in * n_out over the layers
    (the first layer's 12 inputs, not its padding)."""
    return 2 * sum(a * b for a, b in zip(widths[:-1], widths[1:]))
BF16_MFMA_PEAK_TFLOPS = 2500.0


def surrogate_leg(batch=65536, reps=50):
    """Surrogate inference on the matrix cores: the surrogate's network (12
    -> 4 x 256 GELU -> 128; bf16 operands, fp32 accumulation and output) over
    a batch of `batch` seeded feature rows, `reps` forward passes timed with
    HIP events on the network's stream; throughput in samples/s and the
    products' rate against the dense bf16 MFMA peak (464,896 flops per
    sample)."""
    import numpy as np
    import torch

    from paper_1912_03744_amd import native
    from paper_1912_03744_amd import surrogate as S
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        net = native.MLP(S.WIDTHS, seed=5)
        shift, scale = S.feature_scaling()
        net.set_scaling(shift, scale)
        rng = np.random.default_rng(0)
        lo = np.concatenate([S.BOX_LO, [S.LOGT_LO]])
        hi = np.concatenate([S.BOX_HI, [S.LOGT_HI]])
        x = torch.tensor(rng.uniform(lo, hi, size=(batch, 12)).astype(np.float32), device="cuda")
        y = torch.empty(batch, S.WIDTHS[-1], device="cuda")
        for _ in range(3):
            net.forward(x, y)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            net.forward(x, y)
        ev1.record(stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
    tflops = mlp_flop_per_sample(S.WIDTHS) * batch / (ms * 1e-3) / 1e12
    net.close()
    return {"workload": "surrogate forward pass, 12 -> 4 x 256 (GELU) -> %d, bf16 matrix cores with fp32 "
                        "accumulation, batch %d, seeded inputs over the design box" % (S.WIDTHS[-1], batch),
            "value": batch / (ms * 1e-3), "unit": "samples/s", "ms_per_batch": ms,
            "roofline": {"bound": "mfma", "kernel": "k_mlp_fused (whole network)", "achieved": tflops,
                         "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / BF16_MFMA_PEAK_TFLOPS,
                         "traffic": None}}


def training_leg(batch=4096, steps=300):
    """Surrogate training on the matrix cores: `steps` Adam steps (forward,
    backward, update, bf16 weight refresh) of the surrogate's network on
    batches of `batch` seeded rows, timed with HIP events on the network's
    stream; samples/s and the products' rate (three times the forward's
    flops per sample: forward, input gradient, weight gradient) against the
    dense bf16 MFMA peak."""
    import torch

    from paper_1912_03744_amd import native
    from paper_1912_03744_amd import surrogate as S
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        net = native.MLP(S.WIDTHS, seed=6)
        shift, scale = S.feature_scaling()
        net.set_scaling(shift, scale)
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        X = torch.rand(16 * batch, 12, device="cuda", generator=g)
        Y = torch.rand(16 * batch, S.WIDTHS[-1], device="cuda", generator=g)
        for it in range(20):
            net.train_step(X[(it % 16) * batch:(it % 16 + 1) * batch], Y[(it % 16) * batch:(it % 16 + 1) * batch],
                           1e-3)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for it in range(steps):
            net.train_step(X[(it % 16) * batch:(it % 16 + 1) * batch], Y[(it % 16) * batch:(it % 16 + 1) * batch],
                           1e-3)
        ev1.record(stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
    tflops = 3 * mlp_flop_per_sample(S.WIDTHS) * batch / (ms * 1e-3) / 1e12
    net.close()
    return {"workload": "surrogate training step, 12 -> 4 x 256 (GELU) -> %d, MSE + Adam, batch %d, %d steps, "
                        "seeded rows" % (S.WIDTHS[-1], batch, steps),
            "value": batch / (ms * 1e-3), "unit": "samples/s", "us_per_step": ms * 1e3,
            "roofline": {"bound": "mfma", "kernel": "training step (all kernels)", "achieved": tflops,
                         "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / BF16_MFMA_PEAK_TFLOPS,
                         "traffic": None}}


NL_BYTES_PER_CELL_SOLVE = 32  # per line solve: iterate, current layer and explicit part read, new iterate written


def nonlinear_leg(t_end, cpu_steps, cpu=True):
    """The paper's method proper on its case-study grid (Sec. 5: 1210 x 100
    per-layer cells, T0 = 4.2 held on the top face, erf-smoothed pulse of
    t_per = 0.1, t_src = 0.01, t_trs = 1e-4, xi = 4, zeta = 2), with the
    synthetic temperature laws of workloads.case_study_laws: the simple
    iteration of each half step (eps = 1e-7, at most 10 solves, halving
    beyond) and the step rule of Sec. 4 (t_trs/1000 in transitions, t_src/100
    elsewhere), from T0 up to t_end in one adi_nl_run call (persistent
    cooperative kernel).  Throughput counts active cells times accepted
    steps; the kernel's algorithmic bytes are 32 B per active cell and line
    solve (solves of both half steps)."""
    import numpy as np
    import torch

    from paper_1912_03744_amd import native
    from paper_1912_03744_amd import workloads as W
    s = W.case_study()
    laws = W.case_study_laws()
    p = native.Problem.from_spec(s)
    p.set_laws(*laws)
    p.set_pulse("erf", *W.CASE_STUDY_PULSE)
    p.set_iteration(1e-7, 10, 1e-14)
    active = int(np.count_nonzero(p.region_map() != 255))
    p.set_field(None, W.CASE_STUDY_T0)
    p.nl_run(2e-6)            # warm-up: kernel set-up, occupancy, first launch
    p.set_field(None, W.CASE_STUDY_T0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = p.nl_run(t_end)
    wall = time.perf_counter() - t0
    T = p.read_field()
    solves = rep["solves_r"] + rep["solves_z"]
    achieved = NL_BYTES_PER_CELL_SOLVE * active * solves / wall / 1e9
    out = {"workload": "case-study cell of Sec. 5, 1210x100 per-layer grid, synthetic laws, erf pulse "
                       "(t_per 0.1, t_src 0.01, t_trs 1e-4), simple iteration eps 1e-7, step rule of Sec. 4, "
                       "t = 0 to %g" % t_end,
           "value": active * rep["steps"] / wall, "unit": "cell-updates/s", "seconds": wall,
           "steps": rep["steps"], "rejected": rep["rejected"], "solves_r": rep["solves_r"],
           "solves_z": rep["solves_z"], "us_per_step": wall * 1e6 / max(1, rep["steps"]),
           "us_per_solve": wall * 1e6 / max(1, solves), "active_cells": active,
           "t_max": float(np.nanmax(T)), "min_margin": rep["min_margin"],
           "roofline": {"bound": "hbm", "kernel": "nl_run", "achieved": achieved, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "note": "whole persistent launch (line solves, grid-wide waits, step control) over "
                                "its wall time"}}
    p.close()
    if cpu:
        import oracle
        P = oracle.NonlinearProblem(s.geom, s.nr, s.nz, s.h, s.t_inf, s.k, s.rhoc, s.q, s.r_faces, s.z_faces)
        P.set_laws(*laws)
        t0 = time.perf_counter()
        r = P.nl_run(P.initial(W.CASE_STUDY_T0), 0.0, 1.0, kind="erf", pulse_args=W.CASE_STUDY_PULSE, eps=1e-7,
                     iter_max=10, tau_min=1e-14, max_steps=cpu_steps)
        sec = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": active * r["steps"] / sec, "unit": "cell-updates/s", "cores": 1,
                               "kind": "oracle", "seconds": round(sec, 3),
                               "sample": "the first %d steps of the same run (inside the first switch-on "
                                         "transition, %d + %d line solves), single-threaded C -O2"
                                         % (r["steps"], r["solves_r"], r["solves_z"])}
    return out


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--counter-workload":
        counter_workload(0, batch=sys.argv[2:3] == ["batch"])
        return
    if len(sys.argv) > 2 and sys.argv[1] == "--summarize-counters":
        summarize_counters(sys.argv[2], batch=sys.argv[3:4] == ["batch"])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10_000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--graph-steps", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--cpu-threaded-steps", type=int, default=100)
    ap.add_argument("--cpu-batch-steps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-n", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--batch-only", metavar="R,NW,BPC", default=None,
                    help="run only the batch, in this launch shape (no autotuning), and print its figures")
    ap.add_argument("--no-nonlinear", action="store_true")
    ap.add_argument("--nonlinear-t", type=float, default=0.1)
    ap.add_argument("--cpu-nonlinear-steps", type=int, default=400)
    ap.add_argument("--nonlinear-only", action="store_true",
                    help="run only the nonlinear case-study leg and print its figures")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="run only the surrogate inference leg and print its figures")
    ap.add_argument("--training-only", action="store_true",
                    help="run only the surrogate training leg and print its figures")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1912_03744_amd import native
    from paper_1912_03744_amd import workloads as W

    torch.cuda.set_device(0)
    if args.surrogate_only:
        print(json.dumps(surrogate_leg()), flush=True)
        return
    if args.training_only:
        print(json.dumps(training_leg()), flush=True)
        return
    if args.nonlinear_only:
        print(json.dumps(nonlinear_leg(args.nonlinear_t, args.cpu_nonlinear_steps, cpu=not args.no_cpu)),
              flush=True)
        return
    if args.batch_only:
        shape = tuple(int(x) for x in args.batch_only.split(","))
        print(json.dumps(batch_leg(args.batch_n, args.batch_steps, tune=False, shape=shape)), flush=True)
        return
    spec = W.production(args.seed)
    p = native.Problem.from_spec(spec)
    # launch shapes: the project autotuner (times every compiled shape once,
    # outside the timed region; cached per GPU architecture and grid)
    from paper_1912_03744_amd import autotune
    if not args.no_tune:
        t0 = time.perf_counter()
        tuned = autotune.apply(p, spec.dt, spec.scheme)
        print("bench: autotune %.1f s -> %s r %s z %s" % (time.perf_counter() - t0, tuned["layout"],
              tuned["r"]["shape"], tuned["z"]["shape"]), file=sys.stderr, flush=True)
    p.set_check(100, 1e-9)
    p.set_graph_steps(args.graph_steps)
    active = int(np.count_nonzero(p.region_map() != 255))
    cells = spec.nr * spec.nz
    print("bench: %dx%d, %d active cells, launch r=%s z=%s" % (spec.nr, spec.nz, active,
          p.get_launch(0), p.get_launch(1)), file=sys.stderr, flush=True)

    p.step(spec.dt, args.warmup)
    p.read_field()  # synchronises and surfaces latched errors

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.step(spec.dt, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rep = p.energy()  # after the timed region; raises if a periodic check failed
    T = p.read_field()
    assert np.all(np.isfinite(T[~np.isnan(T)]))
    print("bench: %d steps in %.4f s, energy residual %.2e over %d checks"
          % (args.steps, wall, rep["residual"], rep["checks"]), file=sys.stderr, flush=True)

    # dominant kernel: mean launch time of each sweep, HIP events on its stream
    ms_r, ms_z = p.time_sweeps(spec.dt, 200)
    kern, ms = ("sweep_z", ms_z) if ms_z >= ms_r else ("sweep_r", ms_r)
    alg_bytes = BYTES_PER_CELL_HALF_STEP * active
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    traffic = stored_traffic(kern)

    out = {
        "metric": "cell-updates/s per ADI step",
        "value": active * args.steps / wall,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "layered cylinder %dx%d, seeded materials (seed %d), %s, dt=%g, "
                               "%d steps, energy check every 100 steps"
                               % (spec.nr, spec.nz, args.seed, "Peaceman-Rachford", spec.dt, args.steps),
                   "active_cells": active, "cells": cells, "graph_steps": args.graph_steps,
                   "layout": p.layout(), "launch_r": list(p.get_launch(0)),
                   "launch_z": list(p.get_launch(1))},
        "roofline": {"bound": "hbm", "kernel": kern, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "ms_per_launch": {"sweep_r": ms_r, "sweep_z": ms_z},
                     "alg_bytes_per_launch": alg_bytes},
        "cups_all_cells": cells * args.steps / wall,
        "energy_residual": rep["residual"],
    }
    p.close()
    out["single_layout"] = single_layout_leg()
    if not args.no_batch:
        out["batch"] = batch_leg(args.batch_n, args.batch_steps, tune=not args.no_tune)
        print("bench: batch %.3f s, %.3e cell-updates/s" % (out["batch"]["seconds"], out["batch"]["value"]),
              file=sys.stderr, flush=True)
    if not args.no_nonlinear:
        out["nonlinear"] = nonlinear_leg(args.nonlinear_t, args.cpu_nonlinear_steps, cpu=not args.no_cpu)
        print("bench: nonlinear %.3f s, %d steps, %.3e cell-updates/s" % (
            out["nonlinear"]["seconds"], out["nonlinear"]["steps"], out["nonlinear"]["value"]),
            file=sys.stderr, flush=True)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg()
        print("bench: surrogate %.3e samples/s, %.1f TFLOP/s" % (out["surrogate"]["value"],
              out["surrogate"]["roofline"]["achieved"]), file=sys.stderr, flush=True)
        out["surrogate_training"] = training_leg()
        print("bench: surrogate training %.1f us per step, %.1f TFLOP/s" % (
            out["surrogate_training"]["us_per_step"], out["surrogate_training"]["roofline"]["achieved"]),
            file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_steps, args.cpu_threaded_steps)
        if "batch" in out:
            out["batch"]["cpu_baseline"] = batch_cpu_baseline(args.cpu_batch_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
