"""Launch-shape autotuner for the line-solve sweeps and the ragged batch.

Single problems: for each right-hand-side layout (rows, strips of 4
columns) and sweep direction it times every compiled launch shape (cells per
chunk, lines per wave, waves per line, lines per lane, groups per workgroup)
that covers the line length without too much padding, using
adi_time_sweeps (HIP events on the problem's stream); grids small enough for
the LDS-resident time loop time it too (a run of steps in one launch, per
step); it keeps the layout and shapes with the smallest time per step.  Ragged batches: it times the persistent batch kernel (lines per
lane, waves per workgroup, resident workgroups per compute unit) on a short
run of the batch itself with adi_batch_time.  Results are cached in a JSON
file keyed by GPU architecture, problem size (or the batch's size mix) and
scheme: $ADI_AUTOTUNE_CACHE or ~/.cache/adi_autotune.json.
"""
from __future__ import annotations

import json
import os
import time

from . import native

CACHE_ENV = "ADI_AUTOTUNE_CACHE"


def cache_path():
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache",
                                                    "adi_autotune.json")


def _arch():
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def key(nr, nz, scheme):
    return "%s/%dx%d/%s" % (_arch(), nr, nz, scheme)


def candidates(n, nlines, max_pad=2.0, layout="rows", direction=0):
    """Compiled shapes (chunk, lines_per_wave, waves_per_line, lines_per_lane,
    groups_per_block) of a layout covering a line of n cells with at most
    max_pad padding."""
    out = []
    shapes = native.launch_shapes() if layout == "rows" else native.layout_shapes(layout, direction)
    for m, lpw, wpl, r, ngw in shapes:
        G = (64 // lpw) * wpl
        if G * m < n or G * m > max_pad * max(n, 16):
            continue
        if layout == "rows" and lpw * r > max(1, nlines):
            continue
        out.append((m, lpw, wpl, r, ngw))
    return out


def _tune_layout(problem, dt, layout, nlaunch, reps, verbose, log):
    res = {"trials": []}
    dims = {0: (problem.nr, problem.nz), 1: (problem.nz, problem.nr)}
    for d in (0, 1):
        n, nlines = dims[d]
        best = None
        for shape in candidates(n, nlines, layout=layout, direction=d):
            problem.set_launch(d, *shape)
            t = min(problem.time_sweeps(dt, nlaunch)[d] for _ in range(reps))
            res["trials"].append({"layout": layout, "dir": d, "shape": shape, "ms": t})
            if verbose:
                msg = "autotune %s dir %d shape %s: %.4f ms" % (layout, d, shape, t)
                print(msg, flush=True) if log is None else log(msg)
            if best is None or t < best[1]:
                best = (shape, t)
        if best is None:
            return None
        problem.set_launch(d, *best[0])
        res["rz"[d]] = best
    return res


def _time_resident(problem, dt, nlaunch, reps, verbose, log):
    """Time per step of the LDS-resident loop (the whole step, launch
    included, so that it is never favoured over the sweep kernels' own
    durations); its shapes are the rows defaults its check steps use."""
    steps = max(nlaunch, 200)
    t = min(problem.time_sweeps(dt, steps)[0] for _ in range(reps))
    if verbose:
        msg = "autotune resident: %.4f ms per step" % t
        print(msg, flush=True) if log is None else log(msg)
    return {"trials": [{"layout": "resident", "dir": None, "shape": None, "ms": t}],
            "r": (problem.get_launch(0), t), "z": (problem.get_launch(1), 0.0)}


def tune(problem, dt, nlaunch=20, reps=2, verbose=False, log=None):
    """Time every candidate shape of every layout in both directions and set
    the layout and shapes with the smallest r + z time.  Returns {"layout":
    name, "r": (shape, ms), "z": (shape, ms), "trials": [...]}."""
    best, trials = None, []
    for layout in native.LAYOUTS:
        try:
            problem.set_layout(layout)
        except native.AdiError:
            continue
        if layout == "resident":
            res = _time_resident(problem, dt, nlaunch, reps, verbose, log)
        else:
            res = _tune_layout(problem, dt, layout, nlaunch, reps, verbose, log)
        if res is None:
            continue
        trials += res["trials"]
        total = res["r"][1] + res["z"][1]
        if best is None or total < best[0]:
            best = (total, layout, res)
    _, layout, res = best
    problem.set_layout(layout)
    for d in (0, 1):
        problem.set_launch(d, *res["rz"[d]][0])
    return {"layout": layout, "r": res["r"], "z": res["z"], "trials": trials}


def apply(problem, dt, scheme, retune=False, verbose=False, log=None):
    """Set the cached best layout and shapes for this problem size, tuning on
    a miss."""
    db = _load()
    k = key(problem.nr, problem.nz, scheme)
    if not retune and k in db and "layout" in db[k]:
        problem.set_layout(db[k]["layout"])
        for d, name in ((0, "r"), (1, "z")):
            problem.set_launch(d, *db[k][name]["shape"])
        return db[k]
    t0 = time.time()
    r = tune(problem, dt, verbose=verbose, log=log)
    entry = {"layout": r["layout"], "r": {"shape": list(r["r"][0]), "ms": r["r"][1]},
             "z": {"shape": list(r["z"][0]), "ms": r["z"][1]},
             "seconds": time.time() - t0, "trials": len(r["trials"])}
    db = _load()
    db[k] = entry
    _store(db)
    return entry


# compiled batch kernels: (lines per lane, waves per workgroup), 4 lines
# per lane being the strip-layout kernel; resident workgroups per compute
# unit is a launch parameter
BATCH_KERNELS = ((1, 4), (2, 4), (1, 8), (2, 8), (4, 4), (4, 8), (4, 1))
BATCH_BLOCKS_PER_CU = (1, 2, 4)


def batch_key(batch, scheme):
    mix = {}
    for nr, nz in batch.shapes:
        mix["%dx%d" % (nr, nz)] = mix.get("%dx%d" % (nr, nz), 0) + 1
    return "%s/batch%d/%s/%s" % (_arch(), batch.n, ",".join("%s:%d" % kv for kv in sorted(mix.items())),
                                  scheme)


def z_class(nz, classes):
    """z class of the batched sweep launches for columns of nz rows."""
    for c, cl in enumerate(classes):
        if nz <= cl["max_rows"]:
            return c
    raise ValueError("no z class holds %d rows" % nz)


def tune_batch(batch, dt, nsteps=100, verbose=False, log=None):
    """Time every batch launch shape on nsteps steps of the batch itself and
    set the fastest; when that is the batched sweep launches, then time each
    z shape of each size class present (the other classes at their best so
    far) and keep the fastest per class.  Returns {"shape": (R, waves,
    blocks_per_cu), "zshape": [variant per z class], "ms": t, "trials":
    [...]}."""
    def say(msg):
        if verbose:
            print(msg, flush=True) if log is None else log(msg)

    trials, best = [], None
    for c in range(4):
        batch.set_zshape(c, 0)
    for r, nw in BATCH_KERNELS:
        # one wave per workgroup: batched sweep launches, no persistent workgroups
        for bpc in (BATCH_BLOCKS_PER_CU if nw > 1 else (1,)):
            batch.set_launch(r, nw, bpc)
            batch.time(dt, nsteps, 1)  # first call allocates the workgroup scratch
            t = batch.time(dt, nsteps, 1)
            trials.append({"shape": (r, nw, bpc), "ms": t})
            say("autotune batch shape %s: %.3f ms for %d steps" % ((r, nw, bpc), t, nsteps))
            if best is None or t < best[1]:
                best = ((r, nw, bpc), t)
    batch.set_launch(*best[0])
    zshape = [0, 0, 0, 0]
    if best[0][1] == 1:
        from . import native
        classes = native.batch_zshapes()
        t_best = best[1]
        for c in sorted({z_class(nz, classes) for _, nz in batch.shapes}):
            for v in range(1, len(classes[c]["shapes"])):
                batch.set_zshape(c, v)
                t = batch.time(dt, nsteps, 1)
                trials.append({"shape": best[0], "zshape": (c, v), "ms": t})
                say("autotune batch z class %d shape %s: %.3f ms for %d steps"
                    % (c, classes[c]["shapes"][v], t, nsteps))
                if t < t_best:
                    t_best, zshape[c] = t, v
            batch.set_zshape(c, zshape[c])
        best = (best[0], t_best)
    return {"shape": best[0], "zshape": zshape, "ms": best[1], "trials": trials}


def apply_batch(batch, dt, scheme, nsteps=100, retune=False, verbose=False, log=None):
    """Set the cached best batch shape (and z shape per size class) for this
    size mix, tuning on a miss."""
    db = _load()
    k = batch_key(batch, scheme)
    if not retune and k in db and "zshape" in db[k]:
        batch.set_launch(*db[k]["shape"])
        for c, v in enumerate(db[k]["zshape"]):
            batch.set_zshape(c, v)
        return db[k]
    t0 = time.time()
    r = tune_batch(batch, dt, nsteps, verbose=verbose, log=log)
    entry = {"shape": list(r["shape"]), "zshape": list(r["zshape"]), "ms": r["ms"], "steps": nsteps,
             "seconds": time.time() - t0, "trials": len(r["trials"])}
    db = _load()
    db[k] = entry
    _store(db)
    return entry
