"""Host-side pieces of bench.py: the one-GPU guard, launch parsing, the
recorded default launch shapes, and the lookup of committed counter
summaries (which must name the kernel, flags and source they were taken on)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1107_4543_amd import _lib  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_launch_parsing_and_default_shapes_are_valid():
    assert bench.parse_launch("12,64,4,176,1,2") == dict(variant=12, block_x=64, block_y=4, rows=176,
                                                          xcd_remap=1, flags=2)
    with pytest.raises(SystemExit):
        bench.parse_launch("1,2,3")
    d = _lib.lbm_desc()
    d.nx = d.ny = 4096
    d.compute = _lib.LBM_COMPUTE_F32
    d.s_e, d.s_eps, d.s_q, d.s_nu = 1.9, 1.9, 1.9, 1.9
    d.rho0, d.u0x, d.u0y = 1.0, 0.0, 0.0
    d.scale_exp = _lib.LBM_SCALE_AUTO
    for storage, text in bench.DEFAULT_LAUNCH.items():
        d.storage = _lib.STORAGE[storage]
        d.compute = _lib.LBM_COMPUTE_F64 if storage == "f64" else _lib.LBM_COMPUTE_F32
        h = _lib.lbm_create(d, 1 << 32, _lib.lbm_workspace_bytes(d), 0)
        try:
            _lib.lbm_set_launch(h, _lib.lbm_launch(*bench.parse_launch(text).values()))
            assert _lib.lbm_steps_per_launch(_lib.lbm_get_launch(h)) in (5, 6, 7)
        finally:
            _lib.lbm_destroy(h)


def test_profile_lookup_checks_kernel_and_source():
    launch = bench.parse_launch(bench.DEFAULT_LAUNCH["f32"])
    kv = bench.read_profile("waves4096", "f32", launch)
    if kv is not None:                  # committed summary taken on the current source
        assert kv["kernel_source_sha256"] == bench.kernel_source_hash()
        t = bench.read_traffic("waves4096", "f32", launch)
        assert 1.0 <= t / float(kv["algorithmic_bytes_per_launch"]) < 1.5
    other = dict(launch, flags=launch["flags"] ^ 4)
    assert bench.read_traffic("waves4096", "f32", other) is None
    assert bench.read_traffic("waves4096", "f16", launch) is None or os.path.exists(
        os.path.join(ROOT, "profiles", "traffic_step_multi_f16_waves4096.txt"))


def test_pool_roofline_bound_follows_the_steps_per_launch():
    cells, launches, ms = 1 << 20, 10, 2.0
    one = bench.pool_roofline(1, cells, launches, ms)
    assert one["bound"] == "hbm" and one["unit"] == "GB/s"
    us = 1e3 * ms / launches
    assert abs(one["achieved"] - 72 * cells / (us * 1e-6) / 1e9) < 0.1
    assert abs(one["frac"] - one["achieved"] / bench.HBM_PEAK_GBPS) < 1e-4
    multi = bench.pool_roofline(7, cells, launches, ms)
    assert multi["bound"] == "alu" and multi["ops_per_update"] == bench.alg_ops_per_lu("f32", "f32")
    assert multi["algorithmic_ops_per_launch"] == bench.alg_ops_per_lu("f32", "f32") * cells * 7
    assert abs(multi["achieved"] - bench.alg_ops_per_lu("f32", "f32") * cells * 7 / (us * 1e-6) / 1e12) < 0.01
    # with the steps actually run given (67 steps in 10 launches of at most
    # 7), the operations are those of 67 steps, not 70
    part = bench.pool_roofline(7, cells, launches, ms, steps=67)
    assert part["algorithmic_ops_timed"] == bench.alg_ops_per_lu("f32", "f32") * cells * 67
    assert abs(part["achieved"] - bench.alg_ops_per_lu("f32", "f32") * cells * 67 / (ms * 1e-3) / 1e12) < 0.01
    assert abs(multi["peak"] - 39.32) < 0.01 and 0 < multi["frac"] < 1
    assert multi["hbm"]["achieved"] == one["achieved"]
    # the FP64 vector peak is half the FP32 one
    assert bench.ALU_PEAK["f64"] * 2 == bench.ALU_PEAK["f32"]


def test_pool_member_launches_replays_the_chunking():
    shape = bench.parse_pool_shape(bench.DEFAULT_POOL_SHAPE)
    assert shape["steps_per_launch"] == 7 and shape["graph_steps"] == 256
    # 500 steps: chunks 224, 224, 28, 14, 7 (seven-step launches) and one
    # three-step pass
    assert bench.pool_member_launches(shape, 500) == 32 + 32 + 4 + 2 + 1 + 1
    assert bench.pool_member_launches(shape, 7) == 1
    assert bench.pool_member_launches(shape, 3) == 1
    one = dict(shape, steps_per_launch=1)
    assert bench.pool_member_launches(one, 37) == 37


def test_cpu_model_is_read_or_none():
    m = bench.cpu_model()
    assert m is None or (isinstance(m, str) and m)
