"""Host-side logic of bench.py (no GPU): the counter summaries that give
roofline.traffic, and the refusal of more than one GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for k, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Value": v})


@pytest.fixture
def bench(tmp_path, monkeypatch):
    import bench as B
    monkeypatch.setattr(B, "COUNTERS_JSON", str(tmp_path / "sweeps.json"))
    monkeypatch.setattr(B, "BATCH_COUNTERS_JSON", str(tmp_path / "batch.json"))
    return B


def test_sweep_counters_scaled_by_the_copy(bench, tmp_path):
    copy_kib = bench.COUNTER_COPY_BYTES / 1024
    root = tmp_path / "cnt"
    # FETCH reads half the copied bytes, WRITE all of them (as on the chip)
    _csv(str(root / "fetch" / "run_counter_collection.csv"),
         [("void at::neg_kernel(...)", copy_kib / 2)] + [("void adi::k_sweep_zs<5, 8>(adi::StripArgs)", 100.0),
                                                          ("void adi::k_sweep_zs<5, 8>(adi::StripArgs)", 300.0),
                                                          ("void adi::k_sweep_rs<4>(adi::StripArgs)", 50.0)])
    _csv(str(root / "write" / "run_counter_collection.csv"),
         [("void at::neg_kernel(...)", copy_kib)] + [("void adi::k_sweep_zs<5, 8>(adi::StripArgs)", 400.0),
                                                      ("void adi::k_sweep_rs<4>(adi::StripArgs)", 60.0)])
    bench.summarize_counters(str(root))
    rec = json.load(open(bench.COUNTERS_JSON))
    assert rec["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert rec["calibration"]["write_scale"] == pytest.approx(1.0)
    z = rec["kernels"]["sweep_z"]
    assert z["fetch_bytes"] == pytest.approx(200.0 * 1024 * 2)  # mean of the two dispatches, scaled
    assert z["hbm_bytes_per_launch"] == pytest.approx(400 * 1024 + 400 * 1024)
    assert rec["kernels"]["sweep_r"]["hbm_bytes_per_launch"] == pytest.approx(100 * 1024 + 60 * 1024)
    assert rec["source_digest"] == bench.source_digest()
    assert bench.stored_traffic("sweep_z") == pytest.approx(z["hbm_bytes_per_launch"])


def test_batch_counters_summed_per_step(bench, tmp_path):
    copy_kib = bench.COUNTER_COPY_BYTES / 1024
    root = tmp_path / "bcnt"
    kernels = {"void adi::k_bsweep_r<16>(adi::BSweepArgs)": 10.0,
               "_ZN3adi10k_bsweep_rILi64EEEvNS_10BSweepArgsE": 20.0,
               "void adi::k_bsweep_z<4, 2>(adi::BSweepArgs, int)": 30.0,
               "void adi::k_bsweep_z<3, 1>(adi::BSweepArgs, int)": 40.0,
               "adi::k_bsetup(adi::BSweepArgs)": 9999.0}
    rows = [("void at::neg_kernel(...)", copy_kib)]
    for _ in range(3):
        rows += list(kernels.items())
    _csv(str(root / "fetch" / "a_counter_collection.csv"), rows)
    _csv(str(root / "write" / "a_counter_collection.csv"), rows)
    bench.summarize_counters(str(root), batch=True)
    rec = json.load(open(bench.BATCH_COUNTERS_JSON))
    assert sorted(rec["kernels"]) == ["batch_r<16>", "batch_r<64>", "batch_z<3,1>", "batch_z<4,2>"]
    assert rec["kernels"]["batch_z<4,2>"]["dispatches"] == 3
    # every batched-sweep kernel once per step; the set-up kernel is not a step
    assert rec["hbm_bytes_per_step"] == pytest.approx(2 * 100.0 * 1024)
    assert rec["source_digest"] == bench.source_digest(bench.BATCH_SOURCES)
    assert bench.stored_batch_traffic() == pytest.approx(rec["hbm_bytes_per_step"])
    # a reading taken on other sources is not reported
    rec["source_digest"] = "0" * 16
    json.dump(rec, open(bench.BATCH_COUNTERS_JSON, "w"))
    assert bench.stored_batch_traffic() is None


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr
