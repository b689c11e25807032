"""Pins of the linear (von Neumann) analysis and of the oracle's time evolution
against it (no GPU).

* The hydrodynamic eigenvalues of G(k), built from the printed Psi, must
  reproduce at small k the printed modified-equation matrices of Sec. 2.3.1
  (zero mean flow, orders dt^0 and dt^1) and Sec. 2.3.2 (uniform flow, dt^0),
  and the printed sound speed 0.57735.
* A small-amplitude plane wave run through the oracle's nonlinear step must
  decay and rotate per step by those eigenvalues.
"""
import json
import os

import numpy as np
import pytest

import lbm_inputs
import oracle
from oracle import linear

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def printed_B_zero_mean(kx, ky, sigma_e, sigma_nu):
    """B_{,5} terms of order dt^0 and dt^1 at zero mean flow (Sec. 2.3.1)."""
    B0 = 1j * np.array([[0, -kx, -ky], [-kx / 3, 0, 0], [-ky / 3, 0, 0]])
    B1 = np.array([[0, 0, 0],
                   [0, -(kx ** 2) * sigma_e / 3 - (kx ** 2) * sigma_nu / 3 - (ky ** 2) * sigma_nu / 3,
                    -kx * ky * sigma_e / 3],
                   [0, -kx * ky * sigma_e / 3,
                    -(kx ** 2) * sigma_nu / 3 - (ky ** 2) * sigma_e / 3 - (ky ** 2) * sigma_nu / 3]])
    return B0 + B1


def printed_B_uniform_dt0(kx, ky, U, V):
    """B_{,2} term of order dt^0 with uniform flow (Sec. 2.3.2, Eq. uniform-0o)."""
    return 1j * np.array([
        [0, -kx, -ky],
        [-kx / 3 + kx * U ** 2 + ky * U * V, -2 * kx * U - ky * V, -ky * U],
        [-ky / 3 + ky * V ** 2 + kx * U * V, -kx * V, -2 * ky * V - kx * U]])


def _sorted_by_imag(z):
    return z[np.argsort(z.imag)]


@pytest.mark.parametrize("theta", [0.0, np.pi / 6, np.pi / 4, 1.1])
def test_small_k_modes_match_printed_dt0_dt1_matrices(theta):
    s_e, s_eps, s_q, s_nu = 1.2, 1.54, 1.9, 1.1
    sig_e, sig_nu = 1 / s_e - 0.5, 1 / s_nu - 0.5
    k = 2e-3
    kx, ky = k * np.cos(theta), k * np.sin(theta)
    lam, _ = linear.hydrodynamic_modes(kx, ky, s_e, s_eps, s_q, s_nu)
    mu_lbm = _sorted_by_imag(np.log(lam))           # per-step growth exponents
    mu_ns = _sorted_by_imag(np.linalg.eigvals(printed_B_zero_mean(kx, ky, sig_e, sig_nu)))
    # phase: equal to O(k^3); damping: equal to O(k^4) relative to k^2 terms
    assert np.max(np.abs(mu_lbm.imag - mu_ns.imag)) < 5 * k ** 3
    assert np.max(np.abs(mu_lbm.real - mu_ns.real)) < 1e-3 * k ** 2


def test_sound_speed_and_damping_closed_forms():
    # Sec. 5.1 prints c_s = 0.57735; Sec. 4.1 gives Im(omega+-) =
    # -k^2 (nu + eta)/2 and Im(omega^s) = -k^2 nu in 2-D, with nu = sigma_nu/3
    # and eta = sigma_e/3 read from the dt^1 matrix.
    s_e, s_eps, s_q, s_nu = 1.64, 1.54, 1.9, float(linear.s_from_nu(1e-3))
    k = 1e-3
    lam, _ = linear.hydrodynamic_modes(k, 0.0, s_e, s_eps, s_q, s_nu)
    om = 1j * np.log(lam)                            # sorted by Re(omega)
    c = -om[0].real / k, om[2].real / k
    assert abs(c[0] - GOLD["sound_speed"]["c_s"]) < 5e-6 and abs(c[1] - GOLD["sound_speed"]["c_s"]) < 5e-6
    nu, eta = 1e-3, (1 / s_e - 0.5) / 3
    assert abs(om[0].imag / k ** 2 + (nu + eta) / 2) < 1e-4 * (nu + eta)
    assert abs(om[2].imag / k ** 2 + (nu + eta) / 2) < 1e-4 * (nu + eta)
    assert abs(om[1].imag / k ** 2 + nu) < 1e-4 * nu


@pytest.mark.parametrize("U,V,theta", [(0.0577, 0.0, 0.0), (0.1, 0.05, 0.7), (-0.08, 0.03, 2.0)])
def test_uniform_flow_phase_matches_printed_dt0_matrix(U, V, theta):
    s = GOLD["table5"]["A"]
    k = 1e-4
    kx, ky = k * np.cos(theta), k * np.sin(theta)
    lam, _ = linear.hydrodynamic_modes(kx, ky, s["s_e"], s["s_eps"], s["s_q"], s["s_nu"], U, V)
    ph_lbm = np.sort(np.log(lam).imag)
    ph_ns = np.sort(np.linalg.eigvals(printed_B_uniform_dt0(kx, ky, U, V)).imag)
    assert np.max(np.abs(ph_lbm - ph_ns)) < 1e-3 * k
    # closed form: -(U.k_hat +- c_s) k and -(U.k_hat) k
    uk = U * np.cos(theta) + V * np.sin(theta)
    expect = np.sort(-k * np.array([uk - linear.CS, uk, uk + linear.CS]))
    assert np.max(np.abs(ph_lbm - expect)) < 1e-3 * k


def test_lallemand_luo_set_is_linearly_stable():
    s_nu = float(linear.s_from_nu(1e-3))
    assert linear.spectral_radius(1.64, 1.54, 1.9, s_nu, nk=32) <= 1 + 1e-12
    s = GOLD["table5"]["A"]
    assert linear.spectral_radius(s["s_e"], s["s_eps"], s["s_q"], s["s_nu"],
                                  U=0.1 * linear.CS, nk=32) <= 1 + 1e-12


def _project(f, base, mx, nx):
    """Complex Fourier amplitude of population deviations on mode mx along x
    (fields are y-uniform; use row 0)."""
    x = np.arange(nx)
    return ((f[:, 0, :] - base[:, None]) * np.exp(-2j * np.pi * mx * x / nx)[None]).sum(1) * 2 / nx


def test_oracle_plane_wave_phase_and_decay_follow_eigenvalues():
    # The wave workload's recipe on a y-reduced lattice (the field is
    # y-uniform, so one row is exact): per-step ratios of the eigen-coordinates
    # must equal the eigenvalues of G(k).
    nx, mode, A = 256, 4, 1e-4
    s = lbm_inputs.PRESETS["T5A"]
    U0 = 0.1 * lbm_inputs.CS
    rho, ux, uy = lbm_inputs.plane_waves(nx, 1, mode, A, A, U0)
    f = oracle.init(rho, ux, uy)
    base = oracle.init(np.ones((1, 1)), np.full((1, 1), U0), np.zeros((1, 1)))[:, 0, 0]
    k = 2 * np.pi * mode / nx
    rates = [s["s_e"], s["s_eps"], s["s_q"], s["s_nu"]]
    # Decompose on all nine eigenvectors: with rates near 2 the kinetic modes
    # (eigenvalues near 1 - s) decay slowly and must not leak into the fit.
    lam_all, vec_all = linear.eigen(k, 0.0, *rates, U=U0)
    hyd = np.argsort(np.abs(lam_all - 1.0))[:3]
    lam = lam_all[hyd]
    Vinv = np.linalg.inv(vec_all)[hyd]
    coords = []
    steps = 200
    for t in range(steps + 1):
        coords.append(Vinv @ _project(f, base, mode, nx))
        if t < steps:
            f = oracle.run(f, rates, 1)
    c = np.array(coords)                                   # [t, 3]
    checked = 0
    for j in range(3):
        if np.max(np.abs(c[:, j])) < 1e-2 * A:
            continue      # the left-running mode is only excited at O(A^2)
        r = c[1:, j] / c[:-1, j]
        fit = np.mean(r)
        assert abs(np.angle(fit) - np.angle(lam[j])) < 1e-8
        assert abs(abs(fit) - abs(lam[j])) < 1e-8
        checked += 1
    assert checked == 2           # right-running acoustic and shear
