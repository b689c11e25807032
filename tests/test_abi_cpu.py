"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol the header declares, and validates arguments before touching a device.
Nothing here launches a kernel or dereferences device memory."""
import ctypes
import json
import os
import re

import pytest

from paper_1107_4543_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"LBM_API[^;(]*?\b(lbm_\w+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = _lib.load()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # the binding covers the whole header, with the same names
    assert sorted(_lib.SIGNATURES) == names
    for n in names:
        assert callable(getattr(_lib, n))


def desc(**kw):
    d = _lib.lbm_desc()
    d.nx, d.ny = kw.get("nx", 64), kw.get("ny", 48)
    d.storage = kw.get("storage", _lib.LBM_STORE_F32)
    d.compute = kw.get("compute", _lib.LBM_COMPUTE_F32)
    d.s_e, d.s_eps, d.s_q, d.s_nu = kw.get("s", (1.64, 1.54, 1.9, 1.9))
    d.rho0, d.u0x, d.u0y = kw.get("rho0", 1.0), kw.get("u0x", 0.0), 0.0
    d.scale_exp = kw.get("scale_exp", _lib.LBM_SCALE_AUTO)
    d.flags = 0
    return d


def test_s_from_nu_reproduces_table4_viscosities():
    # Table 4 prints s_nu next to nu; s = 1/(3 nu + 1/2) must give back s_nu.
    for g in ("A", "B"):
        row = GOLD["table4"][g]
        assert abs(_lib.lbm_s_from_nu(row["nu"]) - row["s_nu"]) < 5e-7
    assert _lib.lbm_s_from_nu(1e-3) == pytest.approx(1.98807157057654, abs=1e-13)
    assert _lib.lbm_s_from_nu(-1.0) != _lib.lbm_s_from_nu(-1.0)   # NaN


@pytest.mark.parametrize("storage,es", [(0, 8), (1, 4), (2, 2), (3, 2)])
def test_workspace_bytes_formula(storage, es):
    d = desc(nx=100, ny=7, storage=storage, compute=0 if storage == 0 else 1)
    pitch = 128
    buf = (9 * pitch * 7 * es + 255) // 256 * 256
    got = _lib.lbm_workspace_bytes(d)
    assert got > 2 * buf and got - 2 * buf < 200_000


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-3), dict(s=(0.0, 1.5, 1.5, 1.5)), dict(s=(1.5, 2.01, 1.5, 1.5)),
    dict(s=(1.5, 1.5, float("nan"), 1.5)), dict(rho0=0.0), dict(rho0=float("inf")),
    dict(u0x=float("nan")), dict(storage=7), dict(compute=3), dict(storage=1, compute=0),
    dict(storage=2, compute=0), dict(scale_exp=99), dict(nx=70000, ny=70000),
    dict(nx=32768, ny=16384, storage=0, compute=0)])     # one FP64 plane of 4 GiB
def test_invalid_descriptors_are_rejected(bad):
    d = desc(**bad)
    assert _lib.lbm_workspace_bytes(d) == 0
    with pytest.raises(_lib.LbmError) as e:
        _lib.lbm_create(d, 256, 1 << 40, 0)
    assert e.value.status == _lib.LBM_E_INVAL
    assert _lib.lbm_last_error() != ""


def test_largest_planes_are_accepted():
    # one FP32 plane just below 4 GiB (32768 x 32767 cells)
    assert _lib.lbm_workspace_bytes(desc(nx=32768, ny=32767)) > 2 * 9 * 32768 * 32767 * 4


def test_rate_two_is_accepted():
    # Table 4 uses s_eps = 2; the admissible range is read as (0, 2].
    assert _lib.lbm_workspace_bytes(desc(s=(1.99044751, 2.0, 0.00875438872, 1.99044751))) > 0


def test_create_checks_workspace_and_call_order_without_touching_the_device():
    d = desc()
    need = _lib.lbm_workspace_bytes(d)
    fake = 1 << 32          # aligned, never dereferenced by the calls below
    with pytest.raises(_lib.LbmError) as e:
        _lib.lbm_create(d, 0, need, 0)
    assert e.value.status == _lib.LBM_E_INVAL
    with pytest.raises(_lib.LbmError) as e:
        _lib.lbm_create(d, fake + 8, need, 0)
    assert e.value.status == _lib.LBM_E_INVAL
    with pytest.raises(_lib.LbmError) as e:
        _lib.lbm_create(d, fake, need - 1, 0)
    assert e.value.status == _lib.LBM_E_NOMEM
    h = _lib.lbm_create(d, fake, need, 0)
    try:
        assert _lib.lbm_time(h) == 0
        for fn, args in [(_lib.lbm_step, (1,)), (_lib.lbm_read_moments, (8, 8, 8)),
                         (_lib.lbm_read_populations, (8,)), (_lib.lbm_save_state, (8,)),
                         (_lib.lbm_project, (1, 0, 8)), (_lib.lbm_tune, (3,)),
                         (_lib.lbm_set_node_equilibrium, (1, 1, 1.0, 0.0, 0.0))]:
            with pytest.raises(_lib.LbmError) as e:
                fn(h, *args)
            assert e.value.status == _lib.LBM_E_STATE, fn.__name__
        assert _lib.load().lbm_diagnostics(h, (ctypes.c_double * 4)()) == _lib.LBM_E_STATE
        with pytest.raises(_lib.LbmError) as e:
            _lib.lbm_step(h, -1)
        assert e.value.status == _lib.LBM_E_INVAL
        # launch shapes are validated on the host
        assert _lib.lbm_get_launch(h).block_x > 0
        with pytest.raises(_lib.LbmError):
            _lib.lbm_set_launch(h, _lib.lbm_launch(14, 64, 4, 1, 1, 0))
        with pytest.raises(_lib.LbmError):
            _lib.lbm_set_launch(h, _lib.lbm_launch(0, 2048, 1, 1, 1, 0))
        _lib.lbm_set_launch(h, _lib.lbm_launch(2, 64, 4, 2, 0, 0))        # 64 % 4 == 0
        assert _lib.lbm_get_launch(h).as_dict()["variant"] == 2
    finally:
        _lib.lbm_destroy(h)


def test_vector_variants_need_divisible_rows():
    d = desc(nx=66)
    fake = 1 << 32
    h = _lib.lbm_create(d, fake, _lib.lbm_workspace_bytes(d), 0)
    try:
        _lib.lbm_set_launch(h, _lib.lbm_launch(1, 64, 4, 1, 1, 0))         # 66 % 2 == 0
        with pytest.raises(_lib.LbmError):
            _lib.lbm_set_launch(h, _lib.lbm_launch(2, 64, 4, 1, 1, 0))     # 66 % 4 != 0
    finally:
        _lib.lbm_destroy(h)


def test_multi_step_shapes_are_validated_and_report_their_steps():
    d = desc(nx=66)
    fake = 1 << 32
    h = _lib.lbm_create(d, fake, _lib.lbm_workspace_bytes(d), 0)
    try:
        for variant, steps in [(0, 1), (4, 1), (7, 1), (8, 2), (9, 3), (10, 4), (11, 5), (12, 6), (13, 7), (14, 1)]:
            assert _lib.lbm_steps_per_launch(_lib.lbm_launch(variant, 64, 1, 16, 1, 0)) == steps
        _lib.lbm_set_launch(h, _lib.lbm_launch(10, 64, 2, 64, 1, 28))
        _lib.lbm_set_launch(h, _lib.lbm_launch(13, 64, 4, 176, 1, 2))
        assert _lib.lbm_steps_per_launch(_lib.lbm_get_launch(h)) == 7
        _lib.lbm_set_launch(h, _lib.lbm_launch(9, 64, 4, 4096, 0, 7))
        assert _lib.lbm_get_launch(h).variant == 9
        for bad in [(8, 128, 1, 16, 1, 0),      # one wave along x
                    (8, 64, 5, 16, 1, 0),       # at most 4 waves per workgroup
                    (8, 64, 1, 0, 1, 0),        # rows >= 1
                    (10, 64, 1, 4097, 1, 0),    # rows <= 4096
                    (9, 64, 1, 16, 2, 0),       # xcd_remap 0 or 1
                    (10, 64, 1, 16, 1, 30),     # flags 0..29
                    (8, 64, 1, 16, 1, 16),      # skewed pipeline needs T >= 3
                    (10, 64, 1, 16, 1, 17),     # not with non-temporal loads
                    (10, 64, 1, 16, 1, 10),     # one and two rows ahead together
                    (4, 64, 1, 1, 1, 4),        # bit 2 only for several steps per launch
                    (11, 64, 1, 16, 1, 1),      # T = 5: no non-temporal loads
                    (13, 64, 1, 16, 1, 3),      # T = 7: no non-temporal loads
                    (13, 64, 1, 16, 1, 18),     # T = 7: no skewed pipeline
                    (14, 64, 1, 16, 1, 0)]:     # no such variant
            with pytest.raises(_lib.LbmError):
                _lib.lbm_set_launch(h, _lib.lbm_launch(*bad))
        assert _lib.lbm_get_launch(h).variant == 9
    finally:
        _lib.lbm_destroy(h)


def test_step_launch_counts_follow_the_remainder_rule():
    fake = 1 << 32
    d = desc(nx=66)
    h = _lib.lbm_create(d, fake, _lib.lbm_workspace_bytes(d), 0)
    try:
        assert _lib.lbm_step_launches(None, 5) == -1 and _lib.lbm_step_launches(h, -1) == -1
        _lib.lbm_set_launch(h, _lib.lbm_launch(13, 64, 4, 176, 1, 2))          # T = 7
        for n, want in [(0, 0), (1, 1), (2, 1), (6, 1), (7, 1), (8, 2), (9, 2), (12, 2), (2000, 286)]:
            assert _lib.lbm_step_launches(h, n) == want, n
        _lib.lbm_set_launch(h, _lib.lbm_launch(10, 64, 2, 64, 1, 18))          # T = 4, skewed
        # 2 left over: a two-step pass cannot be skewed, so two one-step launches
        assert _lib.lbm_step_launches(h, 6) == 3
        assert _lib.lbm_step_launches(h, 7) == 2                               # 3 left: skewed T = 3
        _lib.lbm_set_launch(h, _lib.lbm_launch(0, 64, 4, 1, 1, 0))
        assert _lib.lbm_step_launches(h, 9) == 9
    finally:
        _lib.lbm_destroy(h)


def test_status_strings():
    for s in (0, -1, -2, -3, -4, -5, 42):
        assert isinstance(_lib.lbm_status_string(s), str) and _lib.lbm_status_string(s)


def test_default_shapes_by_size_and_storage():
    # several steps per launch from 2^19 cells for every storage type, with
    # segments of at least 8 rows; one step below
    fake = 1 << 32
    cases = [("f32", 512, 512, 0), ("f32", 1024, 512, 13), ("f32", 1024, 1024, 13), ("f64", 1024, 1024, 13),
             ("f16", 1024, 511, 0), ("bf16", 723, 723, 0), ("f16", 1024, 512, 12), ("bf16", 1024, 1024, 12),
             ("f16", 2048, 1024, 12), ("bf16", 4096, 4096, 12), ("f32", 4096, 4096, 13)]
    for storage, nx, ny, variant in cases:
        d = desc(nx=nx, ny=ny)
        d.storage = _lib.STORAGE[storage]
        d.compute = _lib.LBM_COMPUTE_F64 if storage == "f64" else _lib.LBM_COMPUTE_F32
        h = _lib.lbm_create(d, fake, _lib.lbm_workspace_bytes(d), 0)
        try:
            c = _lib.lbm_get_launch(h).as_dict()
            assert c["variant"] == variant, (storage, nx, ny, c)
            if variant:
                assert c["block_y"] == 4 and c["flags"] & 32 and c["rows"] >= 8, c
        finally:
            _lib.lbm_destroy(h)
