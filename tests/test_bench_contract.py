"""bench.py's command-line contract on a machine without a GPU, and its roofline
accounting formulas."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_no_gpu_is_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        return
    r = _run("--steps", "1", "--warmup", "0")
    assert r.returncode == 1 and "needs a GPU" in r.stderr and r.stdout == ""


def test_flops_and_bytes_per_field_point_step():
    """474 + 30 log2 Nt flops for three waves (two RK4 half-steps of 228, an FFT pair
    of 5 Nt log2 Nt per field and a 6-flop multiply per field); two waves take two
    thirds of the RK4 and of the per-field terms; 48 B (FP32) and 96 B (FP64) of
    field traffic for three waves."""
    for ln in (10, 14, 16, 20):
        assert bench.flops_per_unit(1 << ln) == 474 + 30 * ln
        assert np.isclose(bench.flops_per_unit(1 << ln, 2), 2 * 228 * 2 / 3 + 2 * 10 * ln + 12)
    assert 3 * bench.BYTES_PER_FIELD["f32"] == 48 and 3 * bench.BYTES_PER_FIELD["f64"] == 96
