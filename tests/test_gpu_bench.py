"""The benchmark's JSON line on a small system: every field of the line the
benchmark prints is present and consistent (the default run uses N = 65536)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_fields():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "4096", "--steps", "2", "--warmup", "1",
           "--cpu-seconds", "0.5", "--energy-seconds", "0.3", "--no-extras"]
    print("running", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline", "sweep", "crackle", "energy_per_interaction"):
        assert key in line, key
    assert line["n_gpus"] == 1 and line["steps"] == 2 and line["warmup"] == 1
    assert line["unit"] == "interactions/s" and line["value"] > 0
    assert line["config"]["workload"] and line["config"]["n"] == 4096
    rf = line["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in rf, key
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s"
    assert 0 < rf["frac"] <= 1 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12
    assert rf["traffic"] is None  # the HBM counters were taken at N = 65536 only
    cb = line["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["sample"]
    assert [r_["n_act"] for r_ in line["sweep"]] == [1, 64, 1024]


def test_bench_split_leg_fields():
    """The split-precision object of the default line, on a small system."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sys.path.insert(0, ROOT)
    import bench
    import nbody_inputs as ni
    n = 2048
    r = bench.split_leg(ni.plummer(n, 2), n, reps=3)
    assert r["median_ms"] > 0 and r["fp64_median_ms"] > 0 and r["interactions_per_s"] > 0
    assert abs(r["speedup_vs_fp64"] - r["fp64_median_ms"] / r["median_ms"]) < 1e-12
    for q in ("a", "j", "s", "phi"):
        e = r["rel_error_vs_fp64_path"][q]
        assert 0 <= e["p50"] <= e["p99"] <= e["max"] < 1e-4, (q, e)
    assert r["integrates"] is False
