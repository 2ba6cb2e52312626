"""The benchmark's output contract, on a small grid: one JSON line with the
required keys, a roofline object and a positive throughput."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line_with_the_contract_keys():
    print("case: bench.py on a 512^2 grid, 6 steps", flush=True)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "512", "--steps", "6", "--warmup", "3", "--forms", "",
           "--cpu-steps", "0", "--batch", "0", "--closure-steps", "0", "--grid3d", "0", "--one-step-steps", "0",
           "--c1-steps", "0", "--c2-steps", "0", "--launch", "224,16,4"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 6 and d["warmup"] == 3 and d["value"] > 0
    assert d["dtype"] == "f32" and d["data"] == "synthetic" and "workload" in d["config"]
    roof = d["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in roof, key
    assert roof["bound"] in ("hbm", "alu") and roof["frac"] > 0
    assert roof["steps_per_launch"] == 3 and roof["launches_timed"] == 2
    assert d["config"]["launch"] == [224, 16, 4]
