"""Pins of the 16-bit storage rounding twin (oracle/storage.py).

* FP16 rounding: every finite binary16 value is kept; every midpoint between
  neighbours goes to the one with an even last bit; one FP64 step off a
  midpoint goes to the nearer neighbour (exhaustive over the format).
* BF16 rounding agrees with PyTorch's CPU float32 -> bfloat16 conversion
  (round to nearest even) on a million values spanning 80 octaves, and sends
  midpoints to even.
* The twin: zero steps is the rounded initial state; an exponent shift of the
  BF16 scale changes nothing (the format is scale invariant away from its
  range limits); every stored value is representable; the density error
  against the unrounded oracle lies below the random-walk rounding bound."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from oracle import linear, storage


def _f16_values():
    bits = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    v = bits.view(np.float16).astype(np.float64)
    return v[np.isfinite(v)]


def test_f16_rounding_is_exhaustively_nearest_even():
    v = _f16_values()
    assert np.array_equal(storage.quantize(v, "f16"), v)
    pos = np.unique(v[v >= 0])                              # 0, subnormals, normals up to 65504
    lo, hi = pos[:-1], pos[1:]
    mid = 0.5 * (lo + hi)                                   # exact in FP64
    even_lo = (lo.astype(np.float16).view(np.uint16) & 1) == 0
    assert np.array_equal(storage.quantize(mid, "f16"), np.where(even_lo, lo, hi))
    assert np.array_equal(storage.quantize(np.nextafter(mid, 0.0), "f16"), lo)
    assert np.array_equal(storage.quantize(np.nextafter(mid, np.inf), "f16"), hi)
    assert np.array_equal(storage.quantize(-mid, "f16"), -np.where(even_lo, lo, hi))
    assert np.array_equal(storage.ulp(lo, "f16"), hi - lo)


def test_bf16_rounding_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(1 << 20) * np.exp2(rng.integers(-40, 40, 1 << 20))).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(storage.quantize(x.astype(np.float64), "bf16"), want)
    # neighbours 1 + k 2^-7 and their midpoints
    lo = 1.0 + np.arange(127) * 2.0 ** -7
    hi = lo + 2.0 ** -7
    k_even = (np.arange(127) % 2) == 0
    assert np.array_equal(storage.quantize(0.5 * (lo + hi), "bf16"), np.where(k_even, lo, hi))
    assert np.array_equal(storage.ulp(lo, "bf16"), hi - lo)


def _pulse():
    nx, ny, A = 48, 40, 1e-3
    rho, ux, uy = lbm_inputs.gaussian_pulse(nx, ny, A, 4.0)
    return oracle.init(rho, ux, uy), A


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_twin_zero_steps_representable_and_within_the_rounding_bound(fmt):
    f0, A = _pulse()
    base = storage.base_state()
    p = storage.scale_exponent(f0, base)
    assert 2.0 ** 12 <= np.max(np.abs(f0 - base)) * 2.0 ** p < 2.0 ** 13
    f, q = storage.run_stored(f0, [1.64, 1.54, 1.9, 1.9], 0, fmt, p, base)
    assert np.array_equal(q, storage.quantize((f0 - base) * 2.0 ** p, fmt))
    steps = 200
    s = [1.64, 1.54, 1.9, float(linear.s_from_nu(1e-3))]
    f, q = storage.run_stored(f0, s, steps, fmt, p, base)
    assert np.array_equal(storage.quantize(q, fmt), q)
    err = np.max(np.abs(oracle.moments(f)[0] - oracle.moments(oracle.run(f0, s, steps))[0])) / A
    u = 2.0 ** -storage.FORMATS[fmt]
    print(fmt, "max|drho|/A", err)
    assert 0 < err <= 3.0 * u * math.sqrt(steps)


def test_twin_bf16_is_scale_invariant():
    f0, _ = _pulse()
    base = storage.base_state()
    p = storage.scale_exponent(f0, base)
    s = [1.64, 1.54, 1.9, 1.95]
    a, _ = storage.run_stored(f0, s, 30, "bf16", p, base)
    b, _ = storage.run_stored(f0, s, 30, "bf16", p + 3, base)
    assert np.array_equal(a, b)
