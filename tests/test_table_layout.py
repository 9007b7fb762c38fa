"""The factor-table index maps of paper_1912_03744_amd/csrc/device.hpp
(pos_at, chk_at), compiled for the host with the test shim of the HIP
device environment: both layouts are one-to-one onto their tables, the plain
layout is field-major, and every field pair of the paired layout (read by
the strip sweeps with one 16-byte load) sits in one aligned slot."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def test_table_index_maps(tmp_path):
    exe = tmp_path / "layout_check"
    subprocess.run(["g++", "-std=c++20", "-O1", "-I", os.path.join(ROOT, "tests", "emu", "shim"),
                    "-I", os.path.join(ROOT, "paper_1912_03744_amd", "csrc"),
                    os.path.join(ROOT, "tests", "emu", "layout_check.cpp"), "-o", str(exe), "-lpthread"],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
