"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (stated with the workload definitions):
* FP64: max |f_gpu - f_oracle| <= 1e-12 max |f_oracle|, and likewise for rho
  and u (u normalised by max |rho|, i.e. momentum-relative).
* FP32: max |rho_gpu - rho_oracle| <= 1e-5 A and max |u_gpu - u_oracle| <=
  1e-5 A_u, with A = max |rho - rho0| and A_u = max |u - u0| of the input.
"""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from oracle import linear

pytestmark = pytest.mark.gpu

LL = lbm_inputs.PRESETS["LL"]
T5A = lbm_inputs.PRESETS["T5A"]


def ll_rates(nu=1e-3):
    return [LL["s_e"], LL["s_eps"], LL["s_q"], float(linear.s_from_nu(nu))]


def t5a_rates():
    return [T5A["s_e"], T5A["s_eps"], T5A["s_q"], T5A["s_nu"]]


def lattice(nx, ny, s, storage="f64", u0=(0.0, 0.0), launch=None, **kw):
    from paper_1107_4543_amd import Lattice
    lat = Lattice(nx, ny, *s, storage=storage, u0=u0, device="cuda:0", **kw)
    if launch is not None:
        lat.set_launch(**launch)
    return lat


def np_(t):
    return t.detach().cpu().numpy()


def check_f64(lat, ref):
    f = np_(lat.populations())
    assert np.max(np.abs(f - ref)) <= 1e-12 * np.max(np.abs(ref))
    r, u, v = (np_(a) for a in lat.moments())
    rr, ur, vr = oracle.moments(ref)
    assert np.max(np.abs(r - rr)) <= 1e-12 * np.max(np.abs(rr))
    assert np.max(np.abs(u - ur)) <= 1e-12 * np.max(np.abs(rr))
    assert np.max(np.abs(v - vr)) <= 1e-12 * np.max(np.abs(rr))


VARIANTS = [dict(variant=0, block_x=64, block_y=4, rows=1, xcd_remap=1),
            dict(variant=0, block_x=32, block_y=8, rows=2, xcd_remap=0),
            dict(variant=1, block_x=64, block_y=2, rows=2, xcd_remap=1),
            dict(variant=2, block_x=64, block_y=4, rows=1, xcd_remap=1),
            dict(variant=3, block_x=128, block_y=1, rows=4, xcd_remap=0),
            dict(variant=0, block_x=128, block_y=2, rows=3, xcd_remap=0, flags=3),
            dict(variant=4, block_x=64, block_y=2, rows=2, xcd_remap=0, flags=2),
            dict(variant=4, block_x=256, block_y=1, rows=1, xcd_remap=1, flags=1),
            dict(variant=5, block_x=64, block_y=4, rows=1, xcd_remap=0, flags=0),
            dict(variant=6, block_x=128, block_y=2, rows=2, xcd_remap=1, flags=1),
            dict(variant=7, block_x=32, block_y=2, rows=1, xcd_remap=0, flags=0)]


@pytest.mark.parametrize("launch", VARIANTS)
def test_pulse64_fp64_matches_oracle(launch):
    # 64 x 64, FP64, Lallemand-Luo set with nu = 1e-3, Gaussian pulse A = 1e-3,
    # half-width 4, centred; 500 steps.
    w = lbm_inputs.WORKLOADS["pulse64"]
    s = ll_rates(w["nu"])
    rho, ux, uy = lbm_inputs.gaussian_pulse(64, 64, w["amplitude"], w["half_width"])
    ref = oracle.run(oracle.init(rho, ux, uy), s, w["steps"])
    lat = lattice(64, 64, s, launch=launch).init(rho, ux, uy).step(w["steps"])
    assert lat.t == w["steps"]
    check_f64(lat, ref)


@pytest.mark.parametrize("nx,ny,steps,u0", [(77, 53, 120, (0.0, 0.0)), (130, 9, 60, (0.05, -0.02)),
                                            (1, 1, 10, (0.0, 0.0)), (1, 17, 25, (0.0, 0.03)),
                                            (23, 1, 25, (0.04, 0.0)), (2, 2, 30, (0.0, 0.0)),
                                            (256, 200, 40, (0.03, 0.01))])
def test_ragged_and_degenerate_sizes_fp64(nx, ny, steps, u0):
    # several tiles and ragged tails (nx not a multiple of 64), single rows and
    # columns, a 1 x 1 lattice (every population streams onto its own cell).
    rng = np.random.default_rng(nx * 1000 + ny)
    rho = 1.0 + 1e-3 * rng.standard_normal((ny, nx))
    ux = u0[0] + 1e-3 * rng.standard_normal((ny, nx))
    uy = u0[1] + 1e-3 * rng.standard_normal((ny, nx))
    s = [1.3, 1.1, 1.7, 1.85]
    ref = oracle.run(oracle.init(rho, ux, uy), s, steps)
    lat = lattice(nx, ny, s, u0=u0).init(rho, ux, uy).step(steps)
    check_f64(lat, ref)


def test_fp64_storage_with_nonzero_base_and_table4_rates():
    # Table 4 group A has s_eps = 2 and s_q close to 0: the edges of the range.
    t4 = lbm_inputs.PRESETS["T4A"]
    s = [t4["s_e"], t4["s_eps"], t4["s_q"], t4["s_nu"]]
    rho, ux, uy = lbm_inputs.gaussian_pulse(96, 64, 1e-3, 5.0, u0=(0.02, 0.01))
    ref = oracle.run(oracle.init(rho, ux, uy), s, 80)
    lat = lattice(96, 64, s, u0=(0.02, 0.01)).init(rho, ux, uy).step(80)
    check_f64(lat, ref)


@pytest.mark.parametrize("launch", VARIANTS[:1] + VARIANTS[3:])
def test_fp32_pulse_matches_oracle_within_1e5_of_amplitude(launch):
    nx, ny, steps, A = 192, 128, 400, 1e-3
    s = ll_rates(1e-3)
    rho, ux, uy = lbm_inputs.gaussian_pulse(nx, ny, A, 6.0, center=(70.3, 50.6), u0=(0.05, 0.0))
    ref = oracle.run(oracle.init(rho, ux, uy), s, steps)
    rr, ur, vr = oracle.moments(ref)
    lat = lattice(nx, ny, s, storage="f32", u0=(0.05, 0.0), launch=launch).init(rho, ux, uy).step(steps)
    r, u, v = (np_(a) for a in lat.moments())
    assert np.max(np.abs(r - rr)) <= 1e-5 * A
    Au = max(np.max(np.abs(ux - 0.05)), np.max(np.abs(uy)), np.max(np.abs(ur - 0.05)))
    assert np.max(np.abs(u - ur)) <= 1e-5 * Au
    assert np.max(np.abs(v - vr)) <= 1e-5 * Au


def test_waves4096_fp32_full_size_matches_row_oracle():
    # 4096 x 4096 FP32, Table 5 group A, acoustic + shear plane waves on a mean
    # flow 0.1 c_s, 2000 steps.  The input does not depend on y, so every row
    # of the exact result equals the oracle run on a 4096 x 1 lattice.
    w = lbm_inputs.WORKLOADS["waves4096"]
    nx, A = w["nx"], w["amplitude"]
    s = t5a_rates()
    rho, ux, uy = lbm_inputs.plane_waves(nx, 1, w["mode"], A, w["shear_amplitude"], w["u0x"])
    ref = oracle.run(oracle.init(rho, ux, uy), s, w["steps"])
    rr, ur, vr = (a[0] for a in oracle.moments(ref))
    lat = lattice(nx, w["ny"], s, storage="f32", u0=(w["u0x"], 0.0))
    R, U, V = (torch.from_numpy(np.broadcast_to(a, (w["ny"], nx)).copy()) for a in (rho, ux, uy))
    lat.init(R, U, V).step(w["steps"])
    r, u, v = lat.moments()
    assert bool((r == r[0:1]).all()) and bool((u == u[0:1]).all()) and bool((v == v[0:1]).all())
    r, u, v = (np_(a[0]) for a in (r, u, v))
    assert np.max(np.abs(r - rr)) <= 1e-5 * A
    Au = max(np.max(np.abs(ux - w["u0x"])), np.max(np.abs(uy)))
    assert np.max(np.abs(u - ur)) <= 1e-5 * Au
    assert np.max(np.abs(v - vr)) <= 1e-5 * Au


@pytest.mark.parametrize("storage,unit", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_sixteen_bit_storage_error_is_within_the_rounding_bound(storage, unit):
    # No tolerance is fixed for 16-bit storage.  Each step rounds nine stored
    # values of size <= A to relative precision u; the errors accumulate as a
    # random walk, so the density error is bounded by C u sqrt(steps) A with a
    # small constant; C = 3 is used (u = 2^-11 for f16, 2^-8 for bf16).
    nx, ny, steps, A = 128, 96, 500, 1e-3
    bound = 3.0 * unit * np.sqrt(steps)
    s = ll_rates(1e-3)
    rho, ux, uy = lbm_inputs.gaussian_pulse(nx, ny, A, 6.0)
    ref = oracle.run(oracle.init(rho, ux, uy), s, steps)
    rr, _, _ = oracle.moments(ref)
    lat = lattice(nx, ny, s, storage=storage).init(rho, ux, uy)
    assert 10 <= lat.scale_exp <= 30           # max|g| ~ 4/9 A ~ 4e-4 -> p = 24
    lat.step(steps)
    r = np_(lat.moments()[0])
    err = np.max(np.abs(r - rr)) / A
    print(f"{storage}: max|drho|/A = {err:.3e}")
    assert err <= bound
    assert err > 0


def test_populations_roundtrip_and_readback_of_init():
    rng = np.random.default_rng(5)
    nx, ny = 70, 33
    rho = 1.0 + 1e-3 * rng.standard_normal((ny, nx))
    ux = 0.02 + 1e-3 * rng.standard_normal((ny, nx))
    uy = 1e-3 * rng.standard_normal((ny, nx))
    s = ll_rates()
    lat = lattice(nx, ny, s, u0=(0.02, 0.0)).init(rho, ux, uy)
    f0 = np_(lat.populations())
    ref0 = oracle.init(rho, ux, uy)
    assert np.max(np.abs(f0 - ref0)) <= 1e-15 * 4
    r, u, v = (np_(a) for a in lat.moments())
    assert np.max(np.abs(r - rho)) < 1e-15 * 4 and np.max(np.abs(u - ux)) < 1e-15 * 4
    # write an oracle state back and continue from it
    ref = oracle.run(ref0, s, 11)
    lat.set_populations(torch.from_numpy(ref))
    lat.step(13)
    check_f64(lat, oracle.run(ref, s, 13))


def test_projection_matches_numpy_fourier_sum():
    rng = np.random.default_rng(9)
    nx, ny = 96, 40
    rho = 1.0 + 1e-3 * rng.standard_normal((ny, nx))
    ux = 0.01 + 1e-3 * rng.standard_normal((ny, nx))
    uy = 1e-3 * rng.standard_normal((ny, nx))
    s = ll_rates()
    lat = lattice(nx, ny, s, u0=(0.01, 0.0)).init(rho, ux, uy).step(7)
    f = np_(lat.populations())
    # the library's own base state, read back from a uniform lattice (g = 0)
    uni = lattice(1, 1, s, u0=(0.01, 0.0)).init(np.ones((1, 1)), np.full((1, 1), 0.01), np.zeros((1, 1)))
    base = np_(uni.populations())[:, 0, 0]
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    # each read-back f = base + g carries one rounding of size ulp(f)/2
    tol_abs = nx * ny * np.spacing(np.max(np.abs(f)))
    for mx, my in [(0, 0), (3, 0), (5, -2), (-7, 11), (95, 39)]:
        frac = ((mx * X) % nx) / nx + ((my * Y) % ny) / ny          # exact phase reduction
        ph = np.exp(-2j * np.pi * frac)
        want = ((f - base[:, None, None]) * ph[None]).sum(axis=(1, 2))
        got = np_(lat.project(mx, my))
        got = got[0::2] + 1j * got[1::2]
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want)) + tol_abs, (mx, my)


@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16"])
def test_mid_size_default_is_several_steps_and_matches_the_oracle(storage):
    # 1100 x 480 = 528,000 cells (at least 2^19): the lattice starts with the
    # several-steps shared-halo shape with short segments (at least 8 rows),
    # whose last strip is partial; 45 steps are six 7-step passes and one
    # 3-step pass (FP32, FP64) or seven 6-step passes and one 3-step pass
    # (FP16, BF16).  Two pulses, one across the periodic seams in x and y.
    nx, ny, steps, A = 1100, 480, 45, 1e-3
    s = t5a_rates()
    rho, ux, uy = lbm_inputs.gaussian_pulse(nx, ny, A, 9.0, center=(300.4, 210.7), u0=(0.05, 0.0))
    rho2, _, _ = lbm_inputs.gaussian_pulse(nx, ny, 0.5 * A, 6.0, center=(1096.2, 2.5))
    rho = rho + (rho2 - 1.0)
    lat = lattice(nx, ny, s, storage=storage, u0=(0.05, 0.0))
    c = lat.launch
    half = storage in ("f16", "bf16")
    assert c["variant"] == (12 if half else 13) and c["flags"] & 32 and c["rows"] >= 8, c
    lat.init(rho, ux, uy).step(steps)
    ref = oracle.run(oracle.init(rho, ux, uy), s, steps)
    if storage == "f64":
        check_f64(lat, ref)
        return
    rr, ur, vr = oracle.moments(ref)
    r, u, v = (np_(a) for a in lat.moments())
    if half:
        # the rounding bound of 16-bit storage, 3 u sqrt(steps) A
        unit = 2.0 ** -11 if storage == "f16" else 2.0 ** -8
        assert np.max(np.abs(r - rr)) <= 3.0 * unit * np.sqrt(steps) * A
        return
    assert np.max(np.abs(r - rr)) <= 1e-5 * A
    Au = max(np.max(np.abs(ux - 0.05)), np.max(np.abs(uy)), np.max(np.abs(ur - 0.05)))
    assert np.max(np.abs(u - ur)) <= 1e-5 * Au
    assert np.max(np.abs(v - vr)) <= 1e-5 * Au


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("nx,ny", [(1 << 20, 3), (3, 1 << 20)])
def test_extreme_aspect_lattices_take_the_default_shape_and_match_the_oracle(storage, nx, ny):
    # 2^20 x 3 and 3 x 2^20 cells (over 2^19: the several-steps default):
    # 4298 strips of one 3-row segment, or one strip whose lanes wrap the
    # 3 columns many times, cut into 768 segments of about 1366 rows; 13
    # steps are a 7-step and a 6-step pass.  Random fields of amplitude A.
    steps, A = 13, 1e-3
    rng = np.random.default_rng(nx + 7 * ny)
    rho = 1.0 + A * rng.standard_normal((ny, nx))
    ux = 0.03 + A * rng.standard_normal((ny, nx))
    uy = A * rng.standard_normal((ny, nx))
    s = t5a_rates()
    lat = lattice(nx, ny, s, storage=storage, u0=(0.03, 0.0))
    c = lat.launch
    assert c["variant"] == 13 and c["flags"] & 32, c
    lat.init(rho, ux, uy).step(steps)
    ref = oracle.run(oracle.init(rho, ux, uy), s, steps)
    if storage == "f64":
        check_f64(lat, ref)
        return
    rr, ur, vr = oracle.moments(ref)
    r, u, v = (np_(a) for a in lat.moments())
    assert np.max(np.abs(r - rr)) <= 1e-5 * A
    assert np.max(np.abs(u - ur)) <= 1e-5 * A
    assert np.max(np.abs(v - vr)) <= 1e-5 * A
