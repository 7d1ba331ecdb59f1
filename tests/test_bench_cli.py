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
from paper_2605_25282_amd import rocprof_summary  # noqa: E402


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
        path = os.path.join(ROOT, "profiles", f"traffic_step_jet5056pair_{prec}.json")
        rec = json.load(open(path))
        assert rec["hashed_sources"] == list(rocprof_summary.STEP_KERNEL_SOURCES)
        got = bench.measured_traffic(prec, "jet5056pair")
        if rec["kernel_source_hash"] == bench.kernel_source_hash():
            assert got == rec["bytes_per_launch"]
            # fetch + write, each scaled by the copy calibration
            assert got == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"], rel=1e-12)
            half = bench.measured_traffic(prec, "jet5056pair", rec["node_updates_per_launch"] / 2)
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


def _counter_db(path, counter, rows):
    """A rocprofv3-style counter database: (dispatch, kernel, value in KiB) per
    dispatch, split over two counter instances as the profiler reports them."""
    import sqlite3
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
              "value real)")
    for d, k, v in rows:
        c.execute("insert into counters_collection values (?, ?, ?, ?)", (d, k, counter, v * 0.25))
        c.execute("insert into counters_collection values (?, ?, ?, ?)", (d, k, counter, v * 0.75))
    c.commit()
    c.close()


def test_counter_summary_calibrates_by_the_last_copy(tmp_path):
    """FETCH_SIZE / WRITE_SIZE are scaled by what they read for the 2 GiB
    calibration copy at the end of the run (here: fetch reads half the copied
    bytes, write all of them), the median over the kernel's dispatches is taken,
    and the record carries the algorithmic bytes and the kernel's source hash."""
    kib = (1 << 31) / 1024.0
    fetch, write = tmp_path / "f.db", tmp_path / "w.db"
    _counter_db(fetch, "FETCH_SIZE", [(1, "vlbm::step_march_kernel<0>", 100.0), (2, "vlbm::step_march_kernel<0>", 130.0),
                                      (3, "vlbm::step_march_kernel<0>", 110.0), (4, "other", 5.0),
                                      (5, "elementwise copy", kib / 2)])
    _counter_db(write, "WRITE_SIZE", [(1, "vlbm::step_march_kernel<0>", 90.0), (2, "vlbm::step_march_kernel<0>", 90.0),
                                      (3, "vlbm::step_march_kernel<0>", 95.0), (4, "copyBuffer", kib)])
    t = rocprof_summary.traffic(str(fetch), str(write), "step_march_kernel")
    assert t["fetch"]["scale"] == pytest.approx(2.0)
    assert t["write"]["scale"] == pytest.approx(1.0)
    assert t["fetch"]["median_bytes"] == pytest.approx(110.0 * 1024 * 2)
    assert t["write"]["median_bytes"] == pytest.approx(90.0 * 1024)
    assert t["bytes_per_launch"] == pytest.approx(110.0 * 2048 + 90.0 * 1024)
    rec = rocprof_summary.record(str(fetch), str(write), "step_march_kernel", "mixed", 1000.0, "w", "s.md")
    assert rec["algorithmic_bytes_per_launch"] == 224.0 * 1000
    assert rec["kernel_source_hash"] == rocprof_summary.kernel_source_hash() == bench.kernel_source_hash()
    assert rec["bytes_per_launch"] == pytest.approx(t["bytes_per_launch"])
    # a run without a calibration copy is refused
    bare = tmp_path / "b.db"
    _counter_db(bare, "FETCH_SIZE", [(1, "vlbm::step_march_kernel<0>", 100.0)])
    with pytest.raises(RuntimeError):
        rocprof_summary.traffic(str(bare), str(write), "step_march_kernel")


def test_committed_default_record_keeps_the_contract():
    """The committed record of the default line has the benchmark's JSON
    contract: the required keys, one GPU, a roofline whose fraction is the
    achieved rate over the 8 TB/s peak and whose traffic is the counted bytes
    of that workload's record, and the oracle baseline with its thread count
    and sample."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "bench_jet5056pair_default.json")))
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in rec, key
    assert rec["n_gpus"] == 1 and rec["unit"] == "GLUPS" and rec["dtype"] == "f64" and rec["higher_is_better"]
    assert rec["config"]["workload"].startswith("jet5056pair")
    roof = rec["roofline"]
    assert roof["bound"] == "hbm" and roof["peak"] == bench.HBM_PEAK_GBS and roof["unit"] == "GB/s"
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], abs=1e-4)
    assert 0.6 <= roof["frac"] < 1.0
    traffic = json.load(open(os.path.join(ROOT, "profiles", "traffic_step_jet5056pair_fp64.json")))
    assert roof["traffic"] == pytest.approx(traffic["bytes_per_launch"], rel=1e-12)
    cpu = rec["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["unit"] == "GLUPS" and cpu["cores"] >= 1 and cpu["sample"]
    assert 0.0 < cpu["value"] < rec["value"]
    mixed = rec["mixed"]
    assert mixed["roofline"]["bytes_per_node_update"] == bench.BYTES_PER_LUP["mixed"]
    assert mixed["speedup_vs_fp64"] == pytest.approx(mixed["value"] / rec["value"], rel=1e-3)
