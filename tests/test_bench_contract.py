"""bench.py's output contract: one JSON line with the metric, the roofline object and the CPU
baseline; one GPU only; algorithmic bytes and the counter-summary lookup."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_bytes_per_node():
    assert bench.bytes_per_node(9, "f32") == 72
    assert bench.bytes_per_node(19, "f32") == 152
    assert bench.bytes_per_node(19, "f16") == 76
    assert bench.bytes_per_node(19, "f32", components=2) == 304


def test_counter_summary_is_used_only_for_the_profiled_kernel_and_tile():
    with open(os.path.join(ROOT, "profiles", "step_counters_foam_3d_f32_f64.json")) as fh:
        d = json.load(fh)
    tile = tuple(d["tile"])
    if d["kernel_hash"] == bench.step_kernel_hash():
        assert bench.traffic_from_profile("foam_3d", "f32", "f64", tile) == d["hbm_bytes_per_launch"]
    other = (tile[0] // 2,) + tile[1:]
    assert bench.traffic_from_profile("foam_3d", "f32", "f64", other) is None
    # each storage type has its own counter summary
    assert bench.traffic_from_profile("foam_3d", "bf16", "f32", tile) is None
    with open(os.path.join(ROOT, "profiles", "step_counters_foam_3d_f16_f32.json")) as fh:
        d16 = json.load(fh)
    assert d16["hbm_bytes_per_launch"] < d["hbm_bytes_per_launch"]
    if d16["kernel_hash"] == bench.step_kernel_hash():
        assert bench.traffic_from_profile("foam_3d", "f16", "f32", tuple(d16["tile"])) == \
            d16["hbm_bytes_per_launch"]


def test_mixture_storage_pairings_are_checked_before_any_gpu_work():
    # FP32 storage pairs with FP64 arithmetic, 16-bit storage with FP32
    for st, comp in (("f16", "f64"), ("f32", "f32")):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload",
                            "mixture_3d", "--storage", st, "--compute", comp],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2
        assert "mixture" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


@pytest.mark.gpu
def test_bench_prints_the_contract_line():
    print("[gpu] bench.py --steps 1 --warmup 0 --cpu-sample-steps 1", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1",
                        "--warmup", "0", "--cpu-sample-steps", "1"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config", "roofline",
              "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["value"] > 0
    assert d["config"]["workload"] == "foam_3d"
    assert d["metric"] == ("Shan-Chen MLUPS & % of HBM roofline; FP16-store/batched vs FP32 at "
                           "fixed err")
    ro = d["roofline"]
    assert ro["bound"] == "hbm" and ro["unit"] == "GB/s" and ro["peak"] == 8000.0
    assert abs(ro["frac"] - ro["achieved"] / ro["peak"]) < 1e-3
    # the measured ceilings: a plain copy, and the step's own memory pattern with its arithmetic
    # left out (flat and marching the step's tiles); the step cannot move data much faster than
    # the marching pattern it is built on
    for k in ("measured_copy_GBps", "measured_pattern_flat_GBps", "measured_pattern_march_GBps"):
        assert ro[k] > 0, k
    assert abs(ro["frac_of_pattern_march"] - ro["achieved"] / ro["measured_pattern_march_GBps"]) < 1e-3
    assert ro["frac_of_pattern_march"] < 1.2
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]
    # the two system patterns of the metric ride on the same line
    pr = d["precision"]
    for k in ("f32 storage / f64 compute", "f16 storage / f32 compute",
              "bf16 storage / f32 compute"):
        assert pr["runs"][k]["MLUPS"] > 0 and 0 < pr["runs"][k]["frac"] < 1
        assert pr["runs"][k]["pattern_march_GBps"] > 0
        assert pr["error_vs_fp64"][k]["rho"] >= 0
    assert pr["error_vs_fp64"]["f32 storage / f64 compute"]["rho"] <= 1e-5
    ba = d["batching"]
    assert ba["MLUPS"] > 0 and ba["one_by_one_MLUPS"] > 0
