"""The batched sweep launches of the ragged batch (set-up kernel, r sweeps
with 4, 2 or 1 row groups per wave, z sweeps in every compiled shape of
each z class, on one, two or three waves per line;
paper_1912_03744_amd/csrc/batch.hpp with the library's own host plan of
workgroup maps), compiled for the host with the stand-in for the HIP device
environment (tests/emu/shim), against the oracle run on every instance
alone: instances of every row-slot width and z shape, odd and tiny grids,
column-class boundaries inside strips, a non-zero ambient temperature and
start value, both schemes."""
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

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")

# (nr, nz): row slots of 16 / 32 / 64 tiles, z chunks of 3 / 4 / 5 cells and
# two waves of 4-cell chunks, and a tiny grid
SIZES = [(40, 100), (100, 250), (150, 300), (61, 400), (7, 9), (33, 150)]


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    exe = tmp_path_factory.mktemp("bemu") / "batch_emu"
    cmd = ["g++", "-std=c++20", "-O1", "-I", os.path.join(ROOT, "tests", "emu", "shim"),
           "-I", os.path.join(ROOT, "paper_1912_03744_amd", "csrc"),
           os.path.join(ROOT, "tests", "emu", "batch_emu.cpp"), "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True)
    return exe


def _specs(scheme):
    base = W.ragged_batch(len(SIZES), master_seed=11, scheme=scheme, dt=2e-3, nsteps=3)
    specs = [s.replace(nr=nr, nz=nz) for s, (nr, nz) in zip(base, SIZES)]
    specs[-1] = specs[-1].replace(t_inf=(0.0, 0.3, -0.2, 0.1), T0=0.3)
    return specs


def _run(emu, tmp_path, specs, scheme, dt, steps, zshape=(0, 0, 0, 0)):
    inp = tmp_path / "batch.txt"
    out = tmp_path / "T.bin"
    with open(inp, "w") as f:
        f.write("%d %d %r %d\n" % (len(specs), 0 if scheme == "pr" else 1, dt, steps))
        for s in specs:
            f.write(" ".join(repr(float(x)) for x in s.geom) + " %d %d\n" % (s.nr, s.nz))
            f.write(" ".join(repr(float(x)) for x in list(s.h) + list(s.t_inf)) + "\n")
            f.write(" ".join(repr(float(x)) for x in list(s.k) + list(s.rhoc) + list(s.q)) + "\n")
            f.write("%r\n" % float(s.T0))
    subprocess.run([str(emu), str(inp), str(out)] + [str(v) for v in zshape], check=True, timeout=600)
    flat = np.fromfile(out)
    fields, o = [], 0
    for s in specs:
        fields.append(flat[o:o + s.nr * s.nz].reshape(s.nz, s.nr))
        o += s.nr * s.nz
    assert o == flat.size
    return fields


# z shape per z class: the defaults, then every other compiled candidate
# (two waves of 3-cell chunks in classes 0-2; one wave of 8-cell chunks and
# three waves of 3-cell chunks in class 3)
ZSHAPES = [("pr", (0, 0, 0, 0)), ("lod", (0, 0, 0, 0)), ("pr", (1, 1, 1, 1)), ("pr", (0, 0, 0, 2))]


@pytest.mark.parametrize("scheme,zshape", ZSHAPES, ids=["%s-z%d%d%d%d" % ((s,) + z) for s, z in ZSHAPES])
def test_batched_sweeps_match_oracle(emu, tmp_path, scheme, zshape):
    specs = _specs(scheme)
    steps, dt = 3, specs[0].dt
    got = _run(emu, tmp_path, specs, scheme, dt, steps, zshape)
    for i, s in enumerate(specs):
        P = oracle.Problem.from_spec(s)
        want, _ = P.step(P.initial(s.T0), scheme, dt, steps)
        act = P.active()
        assert rel_inf(got[i], want, act) <= TOL, (i, s.nr, s.nz)
        assert np.all(got[i][~act] == 0.0)
