"""The acoustic pressure pulse of Sec. 5.2 against its exact solution.

Domain [0, 1]^2 with N nodes per side (dx = dt = 1/N), b = 0.04, t = 0.4
(round(0.4 N) steps), U0 in {0, 0.1}; original rates (Lallemand-Luo,
nu = 1e-5) against the optimised Table 5 group A and B sets; relative L2 error of
the density fluctuation against the exact (linear, inviscid) Bessel-integral
solution.

* With the paper's amplitude eps = 0.01 and N = 64..256: the optimised set
  is more accurate than the original one at every N (the paper's claim), the
  original converges at order about 1, and the optimised one at order about
  2.  The paper reports orders close to 1 for both (Sec. 5.2, Fig. 9, no
  values printed, resolutions and time map not stated).  The reading here:
  dx = dt = 1/N with the rates fixed in lattice units makes a viscous error
  first order and the dispersion error second order; the original set's
  large bulk viscosity dominates its error (order 1, as printed), Table 5's
  does not, so over these resolutions it converges at order 2 (pinned on the
  CPU by test_first_order_of_the_original_set_comes_from_its_bulk_viscosity).
  The assertions encode that reading: order in (0.7, 1.5) for the original,
  above 1.5 for the optimised sets.  (Beyond N = 256 the O(eps)
  nonlinearity, absent from the exact solution, sets a floor near 5e-3.)
* With eps = 1e-3 (linear regime) the optimised set converges at order > 1.5
  up to N = 512.
* The GPU's FP64 errors equal the oracle's (parity), FP32 within 1e-4."""
import functools
import math

import numpy as np
import pytest

import lbm_inputs
import oracle
from oracle import exact_pulse, linear

pytestmark = pytest.mark.gpu

T5A = lbm_inputs.PRESETS["T5A"]
T5B = lbm_inputs.PRESETS["T5B"]
SETS = {"LL": [1.64, 1.54, 1.9, float(linear.s_from_nu(1e-5))],
        "T5A": [T5A["s_e"], T5A["s_eps"], T5A["s_q"], T5A["s_nu"]],
        "T5B": [T5B["s_e"], T5B["s_eps"], T5B["s_q"], T5B["s_nu"]]}


@functools.lru_cache(maxsize=None)
def exact(N, steps, U0, eps):
    return exact_pulse.field(N, N, steps, eps, 0.04 * N, (N / 2, N / 2), u0x=U0)


def errors(N, s, U0, storage, use_oracle=False, eps=0.01):
    from paper_1107_4543_amd import Lattice
    b, steps, c = 0.04 * N, int(round(0.4 * N)), (N / 2, N / 2)
    rho, ux, uy = lbm_inputs.gaussian_pulse(N, N, eps, b, center=c, u0=(U0, 0.0))
    if use_oracle:
        r = oracle.moments(oracle.run(oracle.init(rho, ux, uy), s, steps))[0]
    else:
        lat = Lattice(N, N, *s, storage=storage, u0=(U0, 0.0), device="cuda:0").init(rho, ux, uy).step(steps)
        r = lat.moments()[0].cpu().numpy()
    ex = exact(N, steps, U0, eps)
    full = math.sqrt(np.sum((ex - r) ** 2) / np.sum(ex ** 2))           # as printed (full density)
    fluct = math.sqrt(np.sum((ex - r) ** 2) / np.sum((ex - 1.0) ** 2))  # of the fluctuation
    return full, fluct


def orders(e):
    return [math.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]


@pytest.mark.parametrize("U0", [0.0, 0.1])
def test_pressure_pulse_converges_to_the_exact_solution(U0):
    table = {}
    for name, s in SETS.items():
        table[name] = [errors(N, s, U0, "f64")[1] for N in (64, 128, 256)]
        print(name, U0, ["%.3e" % e for e in table[name]], "orders", [round(o, 2) for o in orders(table[name])])
    for i in range(3):
        assert table["T5A"][i] < table["LL"][i] and table["T5B"][i] < table["LL"][i]
    assert all(0.7 < o < 1.5 for o in orders(table["LL"])), table["LL"]
    assert all(o > 1.5 for o in orders(table["T5A"])), table["T5A"]
    assert all(o > 1.5 for o in orders(table["T5B"])), table["T5B"]


def test_optimised_set_second_order_in_the_linear_regime():
    e = [errors(N, SETS["T5A"], 0.0, "f64", eps=1e-3)[1] for N in (128, 256, 512)]
    print("T5A eps=1e-3", ["%.3e" % x for x in e], "orders", [round(o, 2) for o in orders(e)])
    assert all(o > 1.5 for o in orders(e)), e


def test_gpu_pulse_errors_equal_the_oracle_and_fp32_matches():
    for name, s in SETS.items():
        g = errors(128, s, 0.1, "f64")
        o = errors(128, s, 0.1, "f64", use_oracle=True)
        assert abs(g[1] - o[1]) <= 1e-9 * o[1] and abs(g[0] - o[0]) <= 1e-9 * o[0]
        g32 = errors(128, s, 0.1, "f32")
        assert abs(g32[1] - o[1]) <= 1e-4 * o[1]
