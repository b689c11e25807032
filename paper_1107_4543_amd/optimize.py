"""Free-parameter optimisation of the MRT relaxation rates (Sec. 3.2, App. D).

For zero mean flow, n = 5 and sigma_e = sigma_nu = 0.0025 the paper gives the
cost functions of the dispersion (odd) and dissipation (even) parts of the
perturbation matrix in closed form as polynomials in (sigma_eps, sigma_q)
(App. D); they are written out here.  ``minimize`` searches the admissible
quadrant sigma_eps, sigma_q >= 0 (i.e. s in (0, 2], Sec. 3.2) for the
minimum of F^o (problem Minimization-A) or of F^o + F^e (Minimization-C).
Host-side analysis; it produces relaxation rates for the step kernels.
"""
import math

import numpy as np
from scipy.optimize import minimize as _minimize

# (coefficient, power of sigma_eps, power of sigma_q)
FO_TERMS = [
    (-0.9276312550, 0, 1), (0.1201533868, 1, 0), (7.203744088, 4, 0), (129.3388220, 1, 1),
    (-0.4322246453, 4, 1), (0.01296673935, 3, 3), (-0.00007699001495, 1, 4), (113.4657225, 2, 2),
    (43.21814228, 3, 1), (0.006483369681, 4, 2), (0.01836896999, 1, 3), (-2.155399630, 1, 2),
    (-1.728866164, 3, 2), (0.006483369681, 2, 4), (-0.5121252003, 2, 1), (-1.296718509, 2, 3),
    (0.1080561613, 3, 0), (0.009393468450, 0, 2), (16.02085679, 2, 0), (-0.00006398720339, 0, 3),
    (57.80191535, 0, 0), (0.0000002304635316, 0, 4),
]
FE_TERMS = [
    (0.007225929590, 2, 2), (8.028810655, 2, 0), (0.0000002866536304, 0, 2), (-0.1773049091, 1, 0),
    (-0.00003525193584, 0, 1), (-0.4817286393, 2, 1), (-0.00008580791386, 1, 2),
    (0.008179411071, 1, 1), (0.001159746366, 0, 0),
]


def _poly(terms, se, sq):
    return sum(c * se ** a * sq ** b for c, a, b in terms)


def F_odd(sigma_eps, sigma_q):
    """F^o: dispersion cost (App. D, sigma_e = sigma_nu = 0.0025)."""
    return _poly(FO_TERMS, sigma_eps, sigma_q)


def F_even(sigma_eps, sigma_q):
    """F^e: dissipation cost (App. D, sigma_e = sigma_nu = 0.0025)."""
    return _poly(FE_TERMS, sigma_eps, sigma_q)


def F_total(sigma_eps, sigma_q):
    return F_odd(sigma_eps, sigma_q) + F_even(sigma_eps, sigma_q)


def minimize(cost="odd", starts=None):
    """Minimum of F^o ("odd") or F^o + F^e ("total") over sigma_eps, sigma_q >= 0.
    Returns (sigma_eps, sigma_q, value)."""
    f = F_odd if cost == "odd" else F_total
    if starts is None:
        starts = [(a, b) for a in (0.0, 0.05, 0.5, 2.0) for b in (1.0, 10.0, 50.0, 100.0, 200.0)]
    best = None
    for x0 in starts:
        r = _minimize(lambda v: f(v[0], v[1]), np.array(x0, dtype=float), method="L-BFGS-B",
                      bounds=[(0.0, None), (0.0, None)], options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 2000})
        if best is None or r.fun < best.fun:
            best = r
    return float(best.x[0]), float(best.x[1]), float(best.fun)


def rates_from_sigma(sigma):
    """s = 1 / (sigma + 1/2) (Sec. 2.3)."""
    return 1.0 / (np.asarray(sigma, dtype=np.float64) + 0.5)
