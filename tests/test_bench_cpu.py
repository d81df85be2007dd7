"""Host checks of the benchmark script (no GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_cpu_baseline_fields():
    sys.path.insert(0, ROOT)
    import bench
    import nbody_inputs as ni
    n = 512
    ic = ni.plummer(n, 2)
    r = bench.cpu_baseline(ic, n, 0.3)
    assert r["kind"] == "oracle" and r["unit"] == "interactions/s"
    assert r["value"] > 0 and r["one_core_value"] > 0
    assert r["cores"] >= 1 and isinstance(r["cpu"], str) and r["cpu"]
    assert f"x {n} bodies" in r["sample"]
