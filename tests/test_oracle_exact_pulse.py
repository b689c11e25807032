"""Pins of the exact pressure-pulse solution (Sec. 5.2) against closed forms."""
import math

import numpy as np

from oracle import exact_pulse


def test_initial_time_gives_the_gaussian():
    # Hankel transform pair: int exp(-xi^2/4a) J0(xi eta) xi dxi = 2a exp(-a eta^2)
    b, eps = 5.0, 1e-2
    eta = np.linspace(0.0, 30.0, 301)
    rho = exact_pulse.density(eta, 0.0, eps, b)
    want = 1.0 + eps * np.exp(-math.log(2.0) * eta ** 2 / b ** 2)
    assert np.max(np.abs(rho - want)) < 1e-14


def test_excess_mass_is_conserved():
    # int (rho - rho0) dA = eps pi / alpha at every time
    b, eps = 4.0, 1e-3
    alpha = math.log(2.0) / b ** 2
    for t in (0.0, 10.0, 40.0):
        eta = np.linspace(0.0, exact_pulse.CS * t + 12 * b, 6001)
        r = exact_pulse.density(eta, t, eps, b) - 1.0
        mass = 2 * math.pi * np.trapezoid(r * eta, eta)
        assert abs(mass - eps * math.pi / alpha) < 1e-6 * eps * math.pi / alpha


def test_front_travels_at_the_sound_speed():
    b, eps, t = 3.0, 1e-3, 60.0
    eta = np.linspace(0.0, 60.0, 2401)
    r = exact_pulse.density(eta, t, eps, b) - 1.0
    assert abs(eta[np.argmax(r)] - exact_pulse.CS * t) < b


def test_field_is_advected_by_the_mean_flow():
    f0 = exact_pulse.field(64, 48, 20.0, 1e-3, 4.0, (30.0, 24.0), u0x=0.0)
    f1 = exact_pulse.field(64, 48, 20.0, 1e-3, 4.0, (30.0, 24.0), u0x=0.1)
    assert np.allclose(np.roll(f0, 2, axis=1), f1, atol=1e-15)
