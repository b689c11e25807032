"""GPU invariants that hold at any size, checked bitwise where the arithmetic
is identical: translation, y-uniformity, checkpoint/resume, launch shapes,
tuning leaves the state alone, conservation, and failure reporting."""
import numpy as np
import pytest
import torch

import lbm_inputs
from oracle import linear

pytestmark = pytest.mark.gpu

LL = lbm_inputs.PRESETS["LL"]


def ll_rates(nu=1e-3):
    return [LL["s_e"], LL["s_eps"], LL["s_q"], float(linear.s_from_nu(nu))]


def lattice(nx, ny, s, storage="f32", u0=(0.0, 0.0), **kw):
    from paper_1107_4543_amd import Lattice
    return Lattice(nx, ny, *s, storage=storage, u0=u0, device="cuda:0", **kw)


def fields(nx, ny, seed, u0=(0.0, 0.0)):
    rng = np.random.default_rng(seed)
    return (1.0 + 1e-3 * rng.standard_normal((ny, nx)), u0[0] + 1e-3 * rng.standard_normal((ny, nx)),
            u0[1] + 1e-3 * rng.standard_normal((ny, nx)))


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_translation_invariance_bitwise(storage):
    nx, ny = 128, 96
    rho, ux, uy = fields(nx, ny, 1)
    s = ll_rates()
    a = lattice(nx, ny, s, storage, scale_exp=20 if storage == "f16" else None).init(rho, ux, uy).step(37)
    sh = (5, -9)
    b = lattice(nx, ny, s, storage, scale_exp=20 if storage == "f16" else None)
    b.init(*(np.roll(f, sh, axis=(0, 1)) for f in (rho, ux, uy))).step(37)
    ra = torch.roll(a.populations(), sh, dims=(1, 2))
    assert torch.equal(ra, b.populations())


def test_y_uniform_stays_bitwise_and_large_equals_single_row():
    nx = 1024
    s = [1.99, 1.962820428, 1.992761413, 1.999960001]
    rho, ux, uy = lbm_inputs.plane_waves(nx, 1, 3, 1e-4, 1e-4, 0.0577)
    big = lattice(nx, 256, s, u0=(0.0577, 0.0))
    big.init(*(np.broadcast_to(a, (256, nx)).copy() for a in (rho, ux, uy))).step(100)
    one = lattice(nx, 1, s, u0=(0.0577, 0.0)).init(rho, ux, uy).step(100)
    fb = big.populations()
    assert torch.equal(fb, fb[:, :1].expand_as(fb))
    assert torch.equal(fb[:, :1], one.populations())


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_checkpoint_resume_is_bitwise(storage):
    nx, ny = 96, 80
    rho, ux, uy = fields(nx, ny, 2, (0.03, 0.0))
    s = ll_rates()
    a = lattice(nx, ny, s, storage, u0=(0.03, 0.0)).init(rho, ux, uy).step(60)
    b = lattice(nx, ny, s, storage, u0=(0.03, 0.0)).init(rho, ux, uy).step(30)
    buf, t = b.save_state()
    c = lattice(nx, ny, s, storage, u0=(0.03, 0.0), scale_exp=b.scale_exp).load_state(buf.clone(), t)
    assert c.t == 30
    c.step(30)
    assert torch.equal(a.populations(), c.populations())


@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16"])
def test_all_launch_shapes_give_identical_results(storage):
    nx, ny = 256, 72
    rho, ux, uy = fields(nx, ny, 3, (0.02, 0.01))
    s = ll_rates()
    ref = None
    for launch in [dict(variant=0, block_x=64, block_y=4, rows=1, xcd_remap=1),
                   dict(variant=0, block_x=256, block_y=1, rows=3, xcd_remap=0),
                   dict(variant=1, block_x=64, block_y=1, rows=1, xcd_remap=0),
                   dict(variant=2, block_x=128, block_y=2, rows=2, xcd_remap=1),
                   dict(variant=3, block_x=64, block_y=4, rows=4, xcd_remap=1),
                   dict(variant=0, block_x=64, block_y=2, rows=4, xcd_remap=0, flags=3),
                   dict(variant=2, block_x=64, block_y=2, rows=1, xcd_remap=0, flags=1),
                   dict(variant=4, block_x=128, block_y=4, rows=2, xcd_remap=0, flags=2),
                   dict(variant=4, block_x=1024, block_y=1, rows=1, xcd_remap=1, flags=3),
                   dict(variant=5, block_x=256, block_y=1, rows=2, xcd_remap=0, flags=1),
                   dict(variant=6, block_x=64, block_y=4, rows=1, xcd_remap=1, flags=0),
                   dict(variant=7, block_x=16, block_y=4, rows=3, xcd_remap=0, flags=1),
                   # several steps per launch (25 = passes + left-over single steps)
                   dict(variant=8, block_x=64, block_y=1, rows=16, xcd_remap=0, flags=0),
                   dict(variant=8, block_x=64, block_y=4, rows=64, xcd_remap=1, flags=3),
                   dict(variant=9, block_x=64, block_y=2, rows=7, xcd_remap=0, flags=2),
                   dict(variant=10, block_x=64, block_y=3, rows=100, xcd_remap=1, flags=1),
                   dict(variant=10, block_x=64, block_y=1, rows=1, xcd_remap=0, flags=0),
                   dict(variant=8, block_x=64, block_y=2, rows=32, xcd_remap=1, flags=4),
                   dict(variant=9, block_x=64, block_y=4, rows=5, xcd_remap=0, flags=7),
                   dict(variant=10, block_x=64, block_y=1, rows=128, xcd_remap=1, flags=6),
                   dict(variant=10, block_x=64, block_y=2, rows=9, xcd_remap=1, flags=12),
                   dict(variant=8, block_x=64, block_y=4, rows=1, xcd_remap=0, flags=13),
                   # skewed pipeline
                   dict(variant=10, block_x=64, block_y=1, rows=256, xcd_remap=1, flags=18),
                   dict(variant=9, block_x=64, block_y=3, rows=5, xcd_remap=0, flags=28),
                   dict(variant=10, block_x=64, block_y=4, rows=1, xcd_remap=1, flags=20),
                   # five and six steps per launch
                   dict(variant=11, block_x=64, block_y=1, rows=176, xcd_remap=1, flags=2),
                   dict(variant=12, block_x=64, block_y=4, rows=9, xcd_remap=0, flags=28),
                   # seven steps per launch
                   dict(variant=13, block_x=64, block_y=2, rows=11, xcd_remap=1, flags=2),
                   dict(variant=13, block_x=64, block_y=4, rows=176, xcd_remap=0, flags=12)]:
        lat = lattice(nx, ny, s, storage, u0=(0.02, 0.01))
        lat.set_launch(**launch)
        f = lat.init(rho, ux, uy).step(25).populations()
        if ref is None:
            ref = f
        else:
            assert torch.equal(ref, f), launch


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("nx,ny", [(1, 1), (5, 3), (63, 9), (62, 2), (130, 70), (200, 5), (3, 130)])
def test_several_steps_per_launch_equal_single_steps(storage, nx, ny):
    # tiny, ragged and single-strip lattices; 7 steps leave 1, 1, 3, 2, 1 and
    # 0 single steps over for T = 2 .. 7
    rho, ux, uy = fields(nx, ny, 5, (0.02, -0.01))
    s = ll_rates()
    kw = dict(u0=(0.02, -0.01), scale_exp=22 if storage in ("f16", "bf16") else None)
    ref = lattice(nx, ny, s, storage, **kw).init(rho, ux, uy).step(7).populations()
    for variant, rows, flags in [(8, 4, 0), (9, 1, 3), (10, 64, 2), (8, 3, 4), (9, 16, 5), (10, 2, 6),
                                 (10, 1, 12), (9, 5, 9), (8, 64, 13), (10, 3, 16), (9, 64, 18), (10, 2, 22),
                                 (10, 7, 24), (9, 1, 28), (11, 16, 2), (12, 5, 18), (11, 1, 20), (12, 64, 12),
                                 (13, 3, 0), (13, 64, 2), (13, 1, 12), (13, 9, 4)]:
        lat = lattice(nx, ny, s, storage, **kw)
        lat.set_launch(variant=variant, block_x=64, block_y=2, rows=rows, xcd_remap=1, flags=flags)
        assert lat.steps_per_launch == variant - 6
        lat.init(rho, ux, uy).step(7)
        assert lat.t == 7
        assert torch.equal(lat.populations(), ref), (variant, rows, flags)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("nx,ny", [(1, 1), (5, 3), (63, 9), (130, 70), (200, 5), (3, 130), (260, 33), (520, 40)])
def test_shared_halo_shapes_equal_single_steps(storage, nx, ny):
    # workgroup-shared halo (flag 32): the waves of a workgroup exchange
    # their edge columns through LDS; 1 to 4 waves, T = 4 .. 7, loads one,
    # two or no rows ahead, plain or skewed pipeline (one exchange per
    # stage, or one per row through two alternating buffers); lattices
    # narrower than one wave, wider than a workgroup's strip, ragged and tiny
    rho, ux, uy = fields(nx, ny, 7, (0.02, -0.01))
    s = ll_rates()
    kw = dict(u0=(0.02, -0.01), scale_exp=22 if storage in ("f16", "bf16") else None)
    ref = lattice(nx, ny, s, storage, **kw).init(rho, ux, uy).step(15).populations()
    for variant, block_y, rows, flags in [(13, 4, 168, 34), (13, 4, 7, 32), (13, 1, 16, 40), (13, 2, 3, 34),
                                          (12, 3, 64, 34), (12, 4, 1, 40), (11, 2, 9, 32), (11, 4, 100, 34),
                                          (10, 1, 2, 34), (10, 3, 33, 40),
                                          # skewed pipeline, one exchange per row (flags 48, 50, 56)
                                          (13, 4, 137, 48), (13, 4, 5, 50), (13, 2, 17, 56), (12, 4, 64, 48),
                                          (12, 1, 3, 50), (11, 3, 41, 56), (10, 4, 1, 48), (10, 2, 200, 50)]:
        lat = lattice(nx, ny, s, storage, **kw)
        lat.set_launch(variant=variant, block_x=64, block_y=block_y, rows=rows, xcd_remap=1, flags=flags)
        assert lat.steps_per_launch == variant - 6
        lat.init(rho, ux, uy).step(15)
        assert lat.t == 15
        assert torch.equal(lat.populations(), ref), (variant, block_y, rows, flags)


@pytest.mark.parametrize("compute", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", [(1, 1), (63, 9), (130, 70), (520, 40)])
def test_shared_halo_shapes_equal_single_steps_fp64_storage(compute, nx, ny):
    rho, ux, uy = fields(nx, ny, 8, (0.02, -0.01))
    s = ll_rates()
    kw = dict(u0=(0.02, -0.01), compute=compute)
    ref = lattice(nx, ny, s, "f64", **kw).init(rho, ux, uy).step(15).populations()
    for variant, block_y, rows, flags in [(13, 4, 137, 32), (13, 2, 9, 34), (12, 4, 64, 40), (12, 3, 1, 32)]:
        lat = lattice(nx, ny, s, "f64", **kw)
        lat.set_launch(variant=variant, block_x=64, block_y=block_y, rows=rows, xcd_remap=1, flags=flags)
        lat.init(rho, ux, uy).step(15)
        assert torch.equal(lat.populations(), ref), (variant, block_y, rows, flags)


def test_shared_halo_shapes_are_refused_where_unsupported():
    from paper_1107_4543_amd import _lib
    s = ll_rates()
    lat = lattice(64, 64, s, "f64")
    for bad in [dict(variant=11, flags=34), dict(variant=13, flags=48)]:
        with pytest.raises(_lib.LbmError):
            lat.set_launch(block_x=64, block_y=4, rows=64, xcd_remap=1, **bad)
    lat = lattice(64, 64, s, "f32")
    for bad in [dict(variant=9, block_y=4, flags=34), dict(variant=13, block_y=5, flags=34),
                dict(variant=13, block_y=4, flags=36), dict(variant=13, block_y=4, flags=52),
                dict(variant=9, block_y=4, flags=48)]:
        with pytest.raises(_lib.LbmError):
            lat.set_launch(block_x=64, rows=64, xcd_remap=1, **bad)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_left_over_steps_take_one_shorter_pass(storage):
    # with T = 7, n = 7q + r: q passes, then one r-step pass (r >= 2) or one
    # one-step launch; every split equals n single steps bitwise
    nx, ny = 140, 90
    rho, ux, uy = fields(nx, ny, 6, (0.03, 0.0))
    s = ll_rates()
    kw = dict(u0=(0.03, 0.0), scale_exp=22 if storage == "f16" else None)
    for n in (2, 8, 9, 12, 13, 20):
        ref = lattice(nx, ny, s, storage, **kw).init(rho, ux, uy).step(n).populations()
        lat = lattice(nx, ny, s, storage, **kw)
        lat.set_launch(variant=13, block_x=64, block_y=2, rows=32, xcd_remap=1, flags=2)
        assert lat.launches_for(n) == n // 7 + (1 if n % 7 != 0 else 0)
        lat.init(rho, ux, uy).step(n)
        assert lat.t == n
        assert torch.equal(lat.populations(), ref), n


def test_tune_and_timing_leave_the_state_unchanged():
    nx, ny = 512, 128
    rho, ux, uy = fields(nx, ny, 4)
    s = ll_rates()
    a = lattice(nx, ny, s).init(rho, ux, uy).step(5)
    before = a.populations().clone()
    cfg, us = a.tune(reps=2)
    assert us > 0 and cfg["block_x"] >= 64
    a.time_launches(3)
    assert a.t == 5
    assert torch.equal(before, a.populations())
    a.step(4)
    b = lattice(nx, ny, s).init(rho, ux, uy).step(9)
    assert torch.equal(a.populations(), b.populations())


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_mass_and_momentum_are_conserved(storage):
    nx, ny, A = 256, 256, 1e-3
    rho, ux, uy = lbm_inputs.gaussian_pulse(nx, ny, A, 8.0, u0=(0.04, 0.0))
    lat = lattice(nx, ny, ll_rates(), storage, u0=(0.04, 0.0)).init(rho, ux, uy)
    st0, d0 = lat.diagnostics()
    lat.step(500)
    st1, d1 = lat.diagnostics()
    assert st0 == 0 and st1 == 0 and d1[3] == 0
    # FP64 sum of the initial mass excess: sum A exp(-ln2 d^2/b^2) = A pi b^2 / ln 2
    assert abs(d0[0] - A * np.pi * 64 / np.log(2)) < 1e-6 * d0[0]
    unit = 2.2e-16 if storage == "f64" else 1.2e-7
    tol = 10 * unit * A * np.sqrt(nx * ny * 500)      # random walk of storage rounding
    for k in range(3):
        assert abs(d1[k] - d0[k]) <= tol, (k, d0, d1)


def test_non_finite_input_is_reported():
    from paper_1107_4543_amd import _lib
    nx, ny = 64, 64
    rho, ux, uy = fields(nx, ny, 6)
    rho[10, 20] = np.nan
    lat = lattice(nx, ny, ll_rates()).init(rho, ux, uy)
    st, d = lat.diagnostics()
    assert st == _lib.LBM_E_NONFINITE and d[3] >= 1
    lat.step(3)
    st, d = lat.diagnostics()
    assert st == _lib.LBM_E_NONFINITE and d[3] > 9


def test_unstable_relaxation_set_blows_up_and_is_flagged():
    # A set outside the linear stability region (max |lambda| > 1 at the
    # checkerboard mode) must end in non-finite values that the diagnostics
    # report; the von Neumann screen predicts it.
    s = [1.860, 1.075, 1.312, 1.9169]
    assert linear.spectral_radius(*s, nk=16) > 1.0
    nx = ny = 64
    rho, ux, uy = lbm_inputs.gaussian_pulse(nx, ny, 1e-3, 4.0)
    lat = lattice(nx, ny, s, "f64").init(rho, ux, uy).step(1000)
    st, d = lat.diagnostics()
    from paper_1107_4543_amd import _lib
    assert st == _lib.LBM_E_NONFINITE
