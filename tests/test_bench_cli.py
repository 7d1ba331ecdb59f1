"""Host-side checks of the benchmark's contract: one GPU only, the algorithmic
byte counts, the committed traffic figures and their tie to the step kernel's
sources.  No GPU is used (the GPU-less path must fail with a JSON error)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300)


@pytest.mark.parametrize("n", ["2", "8"])
def test_more_than_one_gpu_is_refused(n):
    r = _run("--gpus", n)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_algorithmic_bytes_per_node_update():
    # FP64: 4 variables x 5 slots, each read once and written once
    assert bench.BYTES_PER_LUP["fp64"] == 2 * 4 * 5 * 8
    # mixed: u (4) and the energy populations (4) in FP64, the other 12 in FP32
    assert bench.BYTES_PER_LUP["mixed"] == 2 * (8 * 8 + 12 * 4)
    assert bench.HBM_PEAK_GBS == 8000.0


def test_traffic_figure_is_tied_to_the_kernel_sources():
    """The committed counter figure is reported only for its own workload and
    only while the step kernel's sources hash to the value recorded with it;
    for another batch size it is scaled by the node updates per launch."""
    for prec in ("fp64", "mixed"):
        path = os.path.join(ROOT, "profiles", f"traffic_step_c5_{prec}.json")
        rec = json.load(open(path))
        assert rec["hashed_sources"] == list(bench.STEP_KERNEL_SOURCES)
        got = bench.measured_traffic(prec, "c5")
        if rec["kernel_source_hash"] == bench.kernel_source_hash():
            assert got == rec["bytes_per_launch"]
            # fetch + write, each scaled by the copy calibration
            assert got == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"], rel=1e-12)
            half = bench.measured_traffic(prec, "c5", rec["node_updates_per_launch"] / 2)
            assert half == pytest.approx(got / 2, rel=1e-12)
            # at least the algorithmic bytes, and not wildly more
            assert 1.0 <= got / rec["algorithmic_bytes_per_launch"] < 1.5
        else:
            assert got is None
        assert bench.measured_traffic(prec, "jet1280") is None


def test_without_a_gpu_the_benchmark_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    r = _run("--steps", "1", "--warmup", "0", "--no-cpu-baseline")
    assert r.returncode == 2
    assert json.loads(r.stdout.strip().splitlines()[-1])["error"] == "no GPU visible"
