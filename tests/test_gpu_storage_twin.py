"""16-bit population storage against the rounding twin (oracle/storage.py).

The GPU collides in FP32 and rounds the post-collision fluctuation, scaled
by 2^p, to FP16 or BF16; the twin collides in FP64 and rounds at the same
points.  Both take the rounding decision in their own precision, so a value
whose FP32 and FP64 post-collision images straddle a rounding midpoint is
stored one unit apart (a "flip"); the probability is about the FP32 error
over the 16-bit spacing, 2^-13 for FP16 and 2^-16 for BF16.

* After initialisation, and after one step from the twin's stored state
  written into the lattice, every stored value equals the twin's, except
  flips, on at most 1 % of the values: adjacent 16-bit values, or, near
  zero where the 16-bit spacing is finer than the FP32 collision error,
  values within that error (8 units of 2^-24 of the largest stored
  magnitude).  Writing a representable state and reading it back is exact.
* Over 500 steps flips spread (the dynamics carry every perturbation without
  damping its rounding consequences), so the two rounding-error fields
  become different samples of one distribution: the GPU's density error
  against the unrounded FP64 oracle must match the twin's, within 25 % in
  the L2 norm and a factor 2 in the maximum.  On the CPU, FP32-sized
  perturbations of the twin move its L2 error by under 12 %, while storing
  with truncation instead of rounding raises it 380-fold (FP16) and 250-fold
  (BF16)."""
import math

import numpy as np
import pytest

import lbm_inputs
import oracle
from oracle import linear, storage

pytestmark = pytest.mark.gpu


def _lattice(nx, ny, s, fmt, u0, p):
    from paper_1107_4543_amd import Lattice
    return Lattice(nx, ny, *s, storage=fmt, u0=u0, scale_exp=p, device="cuda:0")


def _ordinal(q, fmt):
    """Position of representable 16-bit values on the number line (adjacent
    values differ by one; +0 and -0 share 0)."""
    if fmt == "f16":
        u = q.astype(np.float16).view(np.uint16).astype(np.int64)
    else:
        u = (q.astype(np.float32).view(np.uint32) >> 16).astype(np.int64)
    mag = u & 0x7FFF
    return np.where(u >> 15, -mag, mag)


def _compare(x, q, fmt, what, tol):
    """Fraction of stored values that differ from the twin's, and whether
    every difference is a flip: adjacent values, or (for values near zero,
    where the 16-bit spacing is finer than the FP32 error of the collision)
    within tol of each other in stored units."""
    # the readback adds the base in FP64 (2^p * 1e-16 ~ 2e-9 in stored units,
    # far below the spacing of the values present): snap, then compare
    xs = storage.quantize(x, fmt)
    assert np.max(np.abs(xs - x)) < 1e-6
    apart = np.abs(_ordinal(xs, fmt) - _ordinal(q, fmt))
    frac = np.mean(apart > 0)
    ok = (apart <= 1) | (np.abs(xs - q) <= tol)
    print(fmt, what, "differing fraction %.2e" % frac, "max units apart", apart.max(),
          "max distance of the others %.2e (tol %.2e)" % (np.max(np.abs(xs - q)[apart > 1], initial=0.0), tol))
    return frac, bool(ok.all())


@pytest.mark.parametrize("u0", [(0.0, 0.0), (0.05, -0.02)])
@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_stored_values_equal_the_twin_up_to_flips(fmt, u0):
    nx, ny = 130, 70                                 # several tiles, ragged in x
    rng = np.random.default_rng(11)
    rho = 1.0 + 1e-3 * rng.standard_normal((ny, nx))
    ux = u0[0] + 1e-3 * rng.standard_normal((ny, nx))
    uy = u0[1] + 1e-3 * rng.standard_normal((ny, nx))
    s = [1.64, 1.54, 1.9, float(linear.s_from_nu(1e-3))]
    f0 = oracle.init(rho, ux, uy)
    base = storage.base_state(1.0, u0)
    p = storage.scale_exponent(f0, base)
    lat = _lattice(nx, ny, s, fmt, u0, p).init(rho, ux, uy)
    assert lat.scale_exp == p
    scale = 2.0 ** p
    # initialisation rounds the equilibrium fluctuation once
    _, q0 = storage.run_stored(f0, s, 0, fmt, p, base)
    # FP32 collision error, in stored units: a few units of 2^-24 of the
    # largest stored magnitude
    tol = 8 * 2.0 ** -24 * np.max(np.abs(q0))
    frac, ok = _compare((lat.populations().cpu().numpy() - base) * scale, q0, fmt, f"{u0} init", tol)
    assert frac <= 1e-2 and ok
    # writing the twin's stored state is exact
    lat.set_populations(base + q0 / scale)
    frac, ok = _compare((lat.populations().cpu().numpy() - base) * scale, q0, fmt, f"{u0} write", 0.0)
    assert frac == 0
    # one step from the same stored state
    lat.step(1)
    _, q1 = storage.run_stored(base + q0 / scale, s, 1, fmt, p, base)
    frac, ok = _compare((lat.populations().cpu().numpy() - base) * scale, q1, fmt, f"{u0} step", tol)
    assert frac <= 1e-2 and ok


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_storage_error_statistics_match_the_twin(fmt):
    nx, ny, steps, A = 128, 96, 500, 1e-3
    s = [1.64, 1.54, 1.9, float(linear.s_from_nu(1e-3))]
    rho, ux, uy = lbm_inputs.gaussian_pulse(nx, ny, A, 6.0)
    f0 = oracle.init(rho, ux, uy)
    base = storage.base_state()
    p = storage.scale_exponent(f0, base)
    ref = oracle.moments(oracle.run(f0, s, steps))[0]
    twin = oracle.moments(storage.run_stored(f0, s, steps, fmt, p, base)[0])[0]
    lat = _lattice(nx, ny, s, fmt, (0.0, 0.0), p).init(rho, ux, uy).step(steps)
    gpu = lat.moments()[0].cpu().numpy()
    l2 = lambda r: math.sqrt(np.mean((r - ref) ** 2)) / A
    mx = lambda r: np.max(np.abs(r - ref)) / A
    print(fmt, "L2 gpu %.3e twin %.3e" % (l2(gpu), l2(twin)), "max gpu %.3e twin %.3e" % (mx(gpu), mx(twin)))
    assert 0.75 <= l2(gpu) / l2(twin) <= 1.0 / 0.75
    assert 0.5 <= mx(gpu) / mx(twin) <= 2.0
