"""The JSON line bench.py prints for the 4096^2 wave workload: the fields a
measurement harness reads, and a roofline whose bound matches the launch
shape (vector ALU for several steps per launch, HBM for one step)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*extra):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "30", "--warmup", "7",
                        "--cpu-budget", "0", *extra], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_bench_line_for_the_several_steps_default():
    d = run_bench()
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 30 and d["unit"] == "MLUPS" and d["value"] > 0
    assert d["config"]["workload"] == "waves4096" and "cpu_baseline" not in d
    r = d["roofline"]
    assert r["bound"] == "alu" and r["steps_per_launch"] > 1
    assert 0 < r["frac"] <= 1 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    assert r["launches"] == 30 // r["steps_per_launch"] + (1 if 30 % r["steps_per_launch"] else 0)
    # achieved = algorithmic operations per launch over the average launch time
    assert abs(r["achieved"] - r["algorithmic_ops_per_launch"] / (r["avg_launch_us"] * 1e-6) / 1e12) < 0.02
    assert r["hbm"]["bound"] == "hbm" and 0 < r["hbm"]["frac"] < 1


def test_bench_line_for_one_step_per_launch():
    r = run_bench("--launch", "0,512,1,1,0,0")["roofline"]
    assert r["bound"] == "hbm" and r["steps_per_launch"] == 1 and r["launches"] == 30
    assert abs(r["achieved"] - r["algorithmic_bytes_per_launch"] / (r["avg_launch_us"] * 1e-6) / 1e9) < 0.5
