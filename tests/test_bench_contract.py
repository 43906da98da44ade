"""bench.py contract checks that need no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_metric_bytes_formula():
    sys.path.insert(0, ROOT)
    import bench
    # per cell: src + dst (2 n^3), cell metric (7 n^3), three high faces (21 n^2), three penalties
    assert bench.metric_bytes_per_launch(5, 1, 8) == 8 * (2 * 125 + 7 * 125 + 21 * 25 + 3)
    assert bench.metric_bytes_per_launch(5, 10, 4) == 10 * 4 * (9 * 125 + 21 * 25 + 3)


def test_cpu_baseline_reports_cores_and_rate():
    sys.path.insert(0, ROOT)
    import bench
    import dgmf_inputs as inp
    out = bench.cpu_baseline(inp.POISSON_C0, budget_s=0.2)
    assert out["kind"] == "oracle" and out["unit"] == "DoF/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert inp.POISSON_C0.name in out["sample"]
