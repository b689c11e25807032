"""Dispersion and dissipation of the GPU kernels against the von Neumann
analysis (Sec. 4.1), over the wavenumber range and in two directions.

A 128 x 128 lattice carries seven small plane waves at once (|k| from 0.05
to 1.47, along x and along the diagonal); every step the library projects
the population fluctuation on each wave (FP64 on the device) and
``measure_dispersion`` fits every excited eigen-coordinate of G(k).  Each
fitted complex frequency must equal the oracle's eigenvalue of G(k) (built
from the printed Psi): FP64 storage -- every fitted mode, hydrodynamic and
kinetic, within 1e-9 rad per step in phase and 1e-3 of the predicted rate
(plus 1e-10) in growth (measured: 4e-12 and 8e-12); FP32 storage -- the
three hydrodynamic modes, phase within 2e-9 rad per step (measured up to
2.4e-10).  Amplitudes are
1e-7, so mode coupling (second order, and only where two wave vectors add
up to a third) stays below 1e-7 of each wave."""
import math

import numpy as np
import pytest

import lbm_inputs
from oracle import linear

pytestmark = pytest.mark.gpu

WAVES = [(1, 0), (4, 0), (12, 0), (30, 0), (2, 2), (8, 8), (20, 20)]
T5A = lbm_inputs.PRESETS["T5A"]
CASES = {"T5A, U = 0.1 c_s": ([T5A["s_e"], T5A["s_eps"], T5A["s_q"], T5A["s_nu"]], 0.1 * linear.CS, 0.0),
         "LL nu = 1e-3, at rest": ([1.64, 1.54, 1.9, float(linear.s_from_nu(1e-3))], 0.0, 0.0)}


def predicted(m, s, U, V, j):
    lam = np.linalg.eigvals(linear.amplification(m.kx, m.ky, *s, U=U, V=V))
    return lam[np.argmin(np.abs(lam - m.lam[j]))]


def deviation(m, j, want):
    """(phase, growth) per step of the measured eigenvalue relative to want."""
    r = np.exp(-1j * m.omega[j]) / want
    return float(np.angle(r)), float(np.log(np.abs(r)))


@pytest.mark.parametrize("case", list(CASES))
def test_measured_frequencies_equal_the_eigenvalues_fp64(case):
    from paper_1107_4543_amd import vonneumann as vn
    s, U, V = CASES[case]
    res = vn.measure_dispersion(s, WAVES, 128, 128, 400, U, V, storage="f64", amplitude=1e-7)
    fitted = 0
    for m in res:
        hyd = np.argsort(m.conserved)[-3:]
        assert np.all(m.points[hyd] >= 16), (m.wave, m.points)
        for j in np.flatnonzero(m.points):
            want = predicted(m, s, U, V, j)
            dphase, dgrowth = deviation(m, j, want)
            rate = abs(math.log(abs(want)))
            kind = "hydrodynamic" if j in hyd else "kinetic"
            print(case, m.wave, kind, "|lambda| %.4f arg %.4f" % (abs(want), np.angle(want)), "n", m.points[j],
                  "d phase %.1e d growth %.1e" % (dphase, dgrowth))
            assert abs(dphase) <= 1e-9 and abs(dgrowth) <= 1e-3 * rate + 1e-10
            fitted += 1
    assert fitted >= 3 * len(WAVES)


def test_measured_hydrodynamic_phases_fp32():
    from paper_1107_4543_amd import vonneumann as vn
    s, U, V = CASES["T5A, U = 0.1 c_s"]
    res = vn.measure_dispersion(s, WAVES, 128, 128, 400, U, V, storage="f32", amplitude=1e-7)
    for m in res:
        for j in np.argsort(m.conserved)[-3:]:
            assert m.points[j] >= 16
            dphase, _ = deviation(m, j, predicted(m, s, U, V, j))
            print("f32", m.wave, "d phase %.1e" % dphase)
            assert abs(dphase) <= 2e-9
