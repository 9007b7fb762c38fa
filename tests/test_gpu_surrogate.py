"""End-to-end surrogate path at a small scale: labels from the batched FP64
solver, ensemble training on the matrix-core kernels, gate calibration, the
held-out judgement and the screened sweep against the plain and batched
solvers.  Checks the bookkeeping and what the network buys: the screened
sweep evaluates designs faster than the plain per-instance solver, and its
selected designs come back with FP64 solver values."""
import numpy as np
import pytest

from helpers import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_screened_sweep_small():
    from paper_1912_03744_amd import surrogate as S
    res = S.run(n_train=768, n_val=256, n_test=256, n_sweep=8192, n_recall=1024, epochs=4, n_plain=3,
                log=lambda m: print(m, flush=True))
    h, sw = res["heldout"], res["sweep"]
    print(res, flush=True)
    assert 0.0 <= h["gate_pass_rate"] <= 1.0
    # the calibrated gate never keeps a validation design above the target
    assert res["calibration"]["delta"] >= 0.0
    if h["max_err_passed"] is not None:
        assert np.isfinite(h["max_err_passed"])
    assert sw["selected"] == 82 and 0.0 <= sw["recall_at_top"] <= 1.0
    assert -1.0 <= sw["spearman_selected"] <= 1.0
    # what the surrogate gains: screened designs/s beat the plain solver
    assert sw["designs_per_s_screened"] > sw["designs_per_s_plain"]
