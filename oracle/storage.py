"""Rounding twin for 16-bit population storage.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper computes in full precision and says nothing about storage.  The
reading used here: the stored variable is the fluctuation about a uniform
base state, f' = f - f^eq(rho0, U0) (the mean/fluctuation split of Sec. 4.1),
multiplied by a power of two 2^p and rounded to the 16-bit format, to
nearest with ties to even, once at initialisation and once per step on the
post-collision value.  Between roundings everything is the FP64 oracle:
collide in absolute variables, then stream (streaming only moves values, so
it commutes with rounding).

The twin shares its roundings with the GPU path, not its arithmetic: where the
GPU collides in FP32, a post-collision value near a rounding midpoint can
round the other way, and on stable but non-dissipative dynamics such flips
spread until the two rounding-error fields are uncorrelated.  The twin
therefore fixes the distribution of the storage error (its size, and that it
comes from round-to-nearest at scale 2^p), and one step of it fixes each
stored value up to rare one-unit flips.
"""
import numpy as np

from . import collide, init, stream

FORMATS = {"f16": 11, "bf16": 8}      # significant bits, hidden bit included


def quantize(x, storage):
    """Nearest FP16 / BF16 number to each FP64 value, ties to even, returned
    as FP64 (IEEE 754 roundTiesToEven, binary16 and bfloat16 formats)."""
    x = np.asarray(x, dtype=np.float64)
    if storage == "f16":
        # NumPy converts binary64 to binary16 with a single correctly rounded
        # step, subnormals and overflow included.
        return x.astype(np.float16).astype(np.float64)
    if storage == "bf16":
        # bfloat16 keeps binary32's exponent range; at the magnitudes used
        # here (far from 2^-126 and 2^128) rounding to 8 significant bits is
        # the whole conversion.  np.rint rounds half to even.
        m, e = np.frexp(x)                                 # x = m 2^e, 1/2 <= |m| < 1
        return np.ldexp(np.rint(m * 2.0 ** FORMATS["bf16"]), e - FORMATS["bf16"])
    raise ValueError("storage must be 'f16' or 'bf16'")


def ulp(q, storage):
    """Spacing of the 16-bit format at each (representable) value q."""
    bits = FORMATS[storage]
    tiny = 2.0 ** -24 if storage == "f16" else 2.0 ** -133   # subnormal spacing
    q = np.abs(np.asarray(q, dtype=np.float64))
    e = np.frexp(np.where(q > 0, q, 1.0))[1]
    return np.where(q > 0, np.maximum(np.ldexp(1.0, e - bits), tiny), tiny)


def base_state(rho0=1.0, u0=(0.0, 0.0)):
    """f^eq(rho0, U0) as a [9, 1, 1] array (the oracle's own equilibrium)."""
    one = np.ones((1, 1))
    return init(rho0 * one, u0[0] * one, u0[1] * one)


def scale_exponent(f, base):
    """p with 2^p max|f - base| in [2^12, 2^13): the largest stored value
    sits one octave below 2^13, far from the FP16 overflow at 65504."""
    return int(np.floor(np.log2(2.0 ** 13 / np.max(np.abs(f - base)))))


def run_stored(f, s, nsteps, storage, p, base):
    """Pre-collision populations after nsteps steps with the fluctuation
    stored rounded: returns (f, q) with q the stored values (scaled by 2^p,
    in the pre-collision arrangement) and f = base + q 2^-p."""
    scale = 2.0 ** p
    q = quantize((np.asarray(f, dtype=np.float64) - base) * scale, storage)
    for _ in range(int(nsteps)):
        post = collide(base + q / scale, s)
        q = stream(quantize((post - base) * scale, storage))
    return base + q / scale, q
