"""The strip-layout sweep kernels (paper_1912_03744_amd/csrc/strip.hpp and the
lane-block solver of device.hpp), compiled for the host with a stand-in for
the HIP device environment (tests/emu/shim: one thread per lane, workgroup
barriers for LDS, shuffles, DPP row operations and readlane), against the
oracle.  Checks the kernels' logic on the CPU: partial strips and row
groups, strips and row groups that straddle class boundaries, cells outside
the domain, non-zero ambient temperatures, both schemes, one and two waves
per line, strips solved in one pass with two classes' tables (3|1 and
1|3) and strips split between workgroups."""
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
    exe = tmp_path_factory.mktemp("emu") / "strip_emu"
    cmd = ["g++", "-std=c++20", "-O1", "-I", os.path.join(ROOT, "tests", "emu", "shim"),
           "-I", os.path.join(ROOT, "paper_1912_03744_amd", "csrc"),
           os.path.join(ROOT, "tests", "emu", "strip_emu.cpp"), "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True)
    return exe


def _run(emu, tmp_path, s, steps, shape):
    spec = tmp_path / "spec.txt"
    out = tmp_path / "T.bin"
    with open(spec, "w") as f:
        f.write(" ".join(repr(float(x)) for x in s.geom) + " %d %d\n" % (s.nr, s.nz))
        f.write(" ".join(repr(float(x)) for x in list(s.h) + list(s.t_inf)) + "\n")
        f.write(" ".join(repr(float(x)) for x in list(s.k) + list(s.rhoc) + list(s.q)) + "\n")
        f.write("%r %d %d %d %d %d %r\n" % (s.dt, steps, 0 if s.scheme == "pr" else 1, *shape, float(s.T0)))
    subprocess.run([str(emu), str(spec), str(out)], check=True, timeout=300)
    return np.fromfile(out).reshape(s.nz, s.nr)


CASES = [
    ("tiny_3x5_pr", tiny_spec(nr=3, nz=5, scheme="pr", dt=0.02), 4, (1, 3, 1)),
    ("tiny_1x7_lod", tiny_spec(nr=1, nz=7, scheme="lod", dt=0.02), 3, (1, 3, 1)),
    ("tiny_7x12_pr", tiny_spec(nr=7, nz=12, scheme="pr", dt=0.02), 6, (1, 3, 1)),
    ("ambient_61x203_lod", tiny_spec(nr=61, nz=203, scheme="lod", dt=0.02), 5, (1, 5, 1)),
    ("seeded_37x91_pr", W.production(3, nr=37, nz=91).replace(dt=2e-3), 5, (1, 3, 1)),
    ("two_waves_150x333_pr", W.production(3, nr=150, nz=333).replace(dt=2e-3), 3, (1, 5, 2)),
    ("two_waves_r_150x333_lod", tiny_spec(nr=150, nz=333, scheme="lod", dt=0.02), 2, (2, 5, 2)),
    # strips split 1|3 (reverse slot order), 3|1 and 2|2, with ambient films
    ("splits_ambient_128x140_pr",
     W.production(5, nr=128, nz=140).replace(dt=2e-3, t_inf=(0.0, 0.3, -0.2, 0.1), T0=0.2), 4, (1, 3, 1)),
]


@pytest.mark.parametrize("name,spec,steps,shape", CASES, ids=[c[0] for c in CASES])
def test_strip_kernels_match_oracle(emu, tmp_path, name, spec, steps, shape):
    got = _run(emu, tmp_path, spec, steps, shape)
    P = oracle.Problem.from_spec(spec)
    want, _ = P.step(P.initial(spec.T0), spec.scheme, spec.dt, steps)
    act = P.active()
    assert rel_inf(got, want, act) <= TOL
    assert np.all(got[~act] == 0.0)
