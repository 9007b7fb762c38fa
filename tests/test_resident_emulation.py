"""The LDS-resident time loop (paper_1912_03744_amd/csrc/resident.hpp: the
carried right-hand side in LDS, a line per lane and a chunk of it per wave,
the reduced systems solved from both ends, the next right-hand side written
in place), compiled for
the host with the stand-in for the HIP device environment (tests/emu/shim),
against the oracle.  Covers line lengths down to three cells (one chunk
per line), chunks of two to sixteen cells with a partial last chunk, every
boundary class with non-zero ambient temperatures, the cut-out and the
Dirichlet class, both schemes, partial groups of lines, several groups of 64
lines, and runs split over several launches (the carried right-hand side
handed from one launch to the next)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from helpers import rel_inf, tiny_spec
from paper_1912_03744_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = 1e-12

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    exe = tmp_path_factory.mktemp("emu") / "resident_emu"
    cmd = ["g++", "-std=c++20", "-O1", "-w", "-I", os.path.join(ROOT, "tests", "emu", "shim"),
           "-I", os.path.join(ROOT, "paper_1912_03744_amd", "csrc"),
           os.path.join(ROOT, "tests", "emu", "resident_emu.cpp"), "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True)
    return exe


def _run(emu, tmp_path, s, steps, chunk):
    spec = tmp_path / "spec.txt"
    out = tmp_path / "T.bin"
    with open(spec, "w") as f:
        f.write(" ".join(repr(float(x)) for x in s.geom) + " %d %d\n" % (s.nr, s.nz))
        f.write(" ".join(repr(float(x)) for x in list(s.h) + list(s.t_inf)) + "\n")
        f.write(" ".join(repr(float(x)) for x in list(s.k) + list(s.rhoc) + list(s.q)) + "\n")
        f.write("%r %d %d %d %r\n" % (s.dt, steps, 0 if s.scheme == "pr" else 1, chunk, float(s.T0)))
    subprocess.run([str(emu), str(spec), str(out)], check=True, timeout=300)
    return np.fromfile(out).reshape(s.nz, s.nr)


CASES = [
    ("tiny_3x3_pr", tiny_spec(nr=3, nz=3, scheme="pr", dt=0.02), 4, 4),
    ("tiny_4x5_lod", tiny_spec(nr=4, nz=5, scheme="lod", dt=0.02), 3, 1),
    ("tiny_7x12_pr", tiny_spec(nr=7, nz=12, scheme="pr", dt=0.02), 6, 4),
    ("tiny_8x13_lod", tiny_spec(nr=8, nz=13, scheme="lod", dt=0.02), 6, 6),
    ("ambient_37x91_pr", tiny_spec(nr=37, nz=91, scheme="pr", dt=0.02), 5, 2),
    ("seeded_37x91_lod", W.production(3, nr=37, nz=91).replace(dt=2e-3, scheme="lod"), 5, 5),
    ("single_64x160_pr", W.single_layout(scheme="pr"), 7, 3),
    ("single_64x160_lod", W.single_layout(scheme="lod"), 4, 4),
    # many short lines (several groups of 64 lines), and the longest lines
    # (chunks of 16 cells)
    ("wide_200x13_pr",
     W.production(5, nr=200, nz=13).replace(dt=2e-3, t_inf=(0.0, 0.3, -0.2, 0.1), T0=0.2), 3, 2),
    ("tall_5x256_lod", tiny_spec(nr=5, nz=256, scheme="lod", dt=0.01), 3, 3),
]


@pytest.mark.parametrize("name,spec,steps,chunk", CASES, ids=[c[0] for c in CASES])
def test_resident_kernel_matches_oracle(emu, tmp_path, name, spec, steps, chunk):
    got = _run(emu, tmp_path, spec, steps, chunk)
    P = oracle.Problem.from_spec(spec)
    want, _ = P.step(P.initial(spec.T0), spec.scheme, spec.dt, steps)
    act = P.active()
    assert rel_inf(got, want, act) <= TOL
    assert np.all(got[~act] == 0.0)
