"""The JSON line bench.py prints for the 4096^2 wave workload: the fields a
measurement harness reads, a roofline that follows from the line's own
numbers and whose bound matches the launch shape (vector ALU for several
steps per launch, HBM for one step), and the batched and served objects the
default line carries beside it."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ALG_OPS_PER_LU = 70          # FP32 storage and collide: 69 operations and a reciprocal
ALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def run_bench(steps, *extra):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", str(steps), "--warmup", "7",
                        "--cpu-budget", "0", "--batched-steps", "0", "--served-jobs", "0", *extra],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


@pytest.mark.parametrize("steps", [20, 30, 2000])
def test_bench_line_for_the_several_steps_default(steps):
    d = run_bench(steps)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == steps and d["unit"] == "MLUPS" and d["value"] > 0
    assert d["config"]["workload"] == "waves4096" and "cpu_baseline" not in d and "batched" not in d
    assert "serving" not in d
    r = d["roofline"]
    T = r["steps_per_launch"]
    assert r["bound"] == "alu" and T > 1
    assert 0 < r["frac"] <= 1 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    reg = r["timed_region"]
    assert reg["steps"] == steps
    assert reg["launches"] == steps // T + (1 if steps % T else 0) and reg["leftover_launch_steps"] == steps % T
    assert r["launches_timed"] == steps // T
    # the region's ALU figure follows from the line's own MLUPS
    mlups = d["value"]
    assert abs(reg["frac"] - ALG_OPS_PER_LU * mlups * 1e6 / (ALU_PEAK_T * 1e12)) < 1e-3
    # achieved = algorithmic operations of one launch of the dominant kernel
    # over that kernel's own average launch time
    assert r["algorithmic_ops_per_launch"] == ALG_OPS_PER_LU * 4096 * 4096 * T
    assert abs(r["achieved"] - r["algorithmic_ops_per_launch"] / (r["avg_launch_us"] * 1e-6) / 1e12) < 0.02
    # the dominant kernel is at least as fast per step as the whole region:
    # the left-over launch (steps % T steps) reads and writes every
    # population once like a full launch, for fewer steps
    assert r["frac"] >= reg["frac"] * 0.97
    # one-pass equivalent: 72 B per update at the line's update rate
    ope = r["one_pass_equiv"]
    assert ope["bytes_per_update"] == 72
    assert abs(ope["achieved"] - 72 * mlups * 1e6 / 1e9) < 0.5
    assert r["hbm"]["bound"] == "hbm" and 0 < r["hbm"]["frac"] < 1


def test_bench_line_for_one_step_per_launch():
    d = run_bench(30, "--launch", "0,512,1,1,0,0")
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["steps_per_launch"] == 1 and r["launches"] == 30
    assert abs(r["achieved"] - r["algorithmic_bytes_per_launch"] / (r["avg_launch_us"] * 1e-6) / 1e9) < 0.5
    assert abs(r["achieved"] - r["one_pass_equiv"]["achieved"]) < 0.01 * r["achieved"]


def test_bench_line_carries_the_batched_and_served_workloads():
    # last argument wins: the batched run and a short served trace are on
    d = run_bench(14, "--batched-steps", "14", "--served-jobs", "24")
    b = d["batched"]
    assert b["workload"] == "batch256" and b["lattices"] == 256 and b["value"] > 0
    s = d["serving"]
    assert s["workload"] == "serve" and s["jobs"] == 24 and s["rate_jobs_per_s"] == 1000.0
    assert s["served"]["jobs"] == 24 and s["plain"]["jobs"] == 24
    # every served job's final state equals its plain run's (on-device digests)
    assert s["equal_results"] and s["jobs_compared"] == 24 and s["mismatched_jobs"] == []
    assert s["rejected"] == 0 and s["served"]["nonfinite_jobs"] == 0
    for mode in ("served", "plain"):
        m = s[mode]
        assert 0 < m["p50_s"] <= m["p99_s"] <= m["max_s"] and m["aggregate_mlups"] > 0
