"""Host-side checks of the benchmark script (no GPU): its byte accounting and
its refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_step_bytes_of_the_factored_solve_path():
    """Compulsory words per cell of each kernel class: a full step (predictor
    + 2 correctors, each followed by a reduction, a reduced solve and an
    expansion) moves 81.25 words = 325 B a cell with the factored solve."""
    w = bench.alg_words(2)  # the factored (one-ended) solve
    step = w["k_stencil[predictor]"] + 2 * w["k_stencil[corrector]"] + \
        3 * (w["k_reduce"] + w["reduced_solve"] + w["k_expand"])
    assert step == pytest.approx(81.25)
    assert 4 * step == pytest.approx(325.0)
    # the fused-ideal count: 22 words a predictor pass, 21 a corrector pass
    assert bench.FUSED_PRED_B + 2 * bench.FUSED_CORR_B == pytest.approx(256.0)
    # every strategy has an entry; the lane Thomas solve rereads its sweep values
    for solver in range(len(bench.SOLVERS)):
        assert bench.alg_words(solver)["reduced_solve"] >= 1.25
    assert bench.alg_words(1)["reduced_solve"] == pytest.approx(2.25)


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
