"""Host von Neumann analysis (paper_1107_4543_amd/vonneumann.py, Sec. 4.1).

Pinned against the oracle's independent construction (G(k) from the printed
linear collision matrix Psi, Sec. 2.3) and against closed forms: small-k
phase speeds c_s +- U.khat and 0, damping (nu + bulk)/2 k^2 and nu k^2 at
zero mean flow (the linearised isothermal Navier-Stokes modes), mirror
symmetry of the two acoustic branches, continuity of the tracked branches,
symmetries of the stability map and the oracle's spectral radius."""
import math

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import lbm_inputs
from oracle import linear
from paper_1107_4543_amd import stability, vonneumann as vn


def rates(name):
    if name == "LL":
        return [1.64, 1.54, 1.9, float(linear.s_from_nu(1e-3))]
    p = lbm_inputs.PRESETS[name]
    return [p["s_e"], p["s_eps"], p["s_q"], p["s_nu"]]


def test_amplification_equals_the_oracle_built_from_printed_psi():
    rng = np.random.default_rng(3)
    for _ in range(20):
        s = rng.uniform(0.3, 2.0, 4)
        kx, ky = rng.uniform(-math.pi, math.pi, 2)
        U, V = rng.uniform(-0.1, 0.1, 2)
        assert np.max(np.abs(vn.amplification(s, kx, ky, U, V) - linear.amplification(kx, ky, *s, U=U, V=V))) < 1e-14


def test_broadcasting_over_rates_wavenumbers_and_flows():
    rng = np.random.default_rng(4)
    R = rng.uniform(0.5, 2.0, (3, 1, 4))
    k = rng.uniform(-3, 3, (3, 5))
    U = np.array([0.0, 0.05, -0.02])[:, None]
    G = vn.amplification(R, k, -k, U, 0.01)
    assert G.shape == (3, 5, 9, 9)
    for i in range(3):
        for j in range(5):
            assert np.array_equal(G[i, j], vn.amplification(R[i, 0], k[i, j], -k[i, j], U[i, 0], 0.01))


@pytest.mark.parametrize("name", ["LL", "T5A", "T4A"])
@pytest.mark.parametrize("theta", [0.0, math.pi / 4, 0.3])
def test_small_k_modes_are_the_navier_stokes_modes(name, theta):
    s = rates(name)
    k = np.array([1e-3, 2e-3])
    d = vn.dispersion(s, k, theta)
    ns = vn.navier_stokes(k, theta, s)
    for lab in vn.HYDRO:
        om = d.omega[:, d.column(lab)]
        assert np.all(np.abs(om.real - ns[lab].real) <= 1e-6 * k)
        assert np.all(np.abs(om.imag - ns[lab].imag) <= 2e-3 * np.abs(ns[lab].imag))
    assert sorted(d.labels) == sorted(list(vn.HYDRO) + ["kinetic"] * 6)


@pytest.mark.parametrize("theta", [0.0, math.pi / 4])
def test_small_k_phase_speed_with_mean_flow(theta):
    s = rates("T5A")
    U, V = 0.1 * linear.CS, 0.02
    d = vn.dispersion(s, np.array([1e-3]), theta, U, V)
    adv = U * math.cos(theta) + V * math.sin(theta)
    assert abs(d.phase_speed("acoustic+")[0] - (adv + vn.CS)) < 1e-6
    assert abs(d.phase_speed("acoustic-")[0] - (adv - vn.CS)) < 1e-6
    assert abs(d.phase_speed("shear")[0] - adv) < 1e-6


@pytest.mark.parametrize("name", ["LL", "T5A"])
@pytest.mark.parametrize("theta", [0.0, math.pi / 4])
def test_branches_are_continuous_and_mirror_at_rest(name, theta):
    s = rates(name)
    k = np.linspace(1e-3, 0.9 * math.pi, 300)
    d = vn.dispersion(s, k, theta)
    cols = [d.column(lab) for lab in vn.HYDRO]
    om = d.omega[:, cols]
    assert np.max(np.abs(np.diff(om, axis=0))) < 0.05           # steps of dk = 0.0094
    # at rest the two acoustic branches are mirror images (k -> -k) while they
    # propagate.  Along the diagonal the pair meets at an exceptional point and
    # becomes two real (non-propagating) eigenvalues: over a band from
    # k ~ 2.42 with the strongly damped LL rates (overdamped sound), at a
    # single crossing of zero frequency near k ~ 2.51 with Table 5 A.
    a_plus, a_minus = om[:, 2], om[:, 0]
    moving = np.abs(a_plus.real) > 1e-9
    n = int(np.argmin(moving)) if not moving.all() else k.size
    first_stop = {("LL", 0.0): None, ("T5A", 0.0): None, ("LL", math.pi / 4): (2.3, 2.5),
                  ("T5A", math.pi / 4): (2.45, 2.55)}[(name, theta)]
    if first_stop is None:
        assert n == k.size
    else:
        assert n < k.size and first_stop[0] < k[n] < first_stop[1]
    assert np.max(np.abs(a_plus.real + a_minus.real)[:n]) < 1e-9
    assert np.max(np.abs(a_plus.imag - a_minus.imag)[:n]) < 1e-9
    # every eigenvalue is tracked, none lost or duplicated
    ref = np.linalg.eigvals(linear.amplification(k[-1] * math.cos(theta), k[-1] * math.sin(theta), *s))
    dist = np.abs(d.lam[-1][:, None] - ref[None, :])
    rows, cols = linear_sum_assignment(dist)
    assert np.max(dist[rows, cols]) < 1e-10


def test_stability_map_symmetries_and_oracle_radius():
    s = rates("T4A")
    m = vn.stability_map(s, nk=32)
    assert np.max(np.abs(m - m.T)) < 1e-12                                  # x <-> y
    assert np.max(np.abs(m - np.roll(m[::-1, ::-1], 1, axis=(0, 1)))) < 1e-12   # k -> -k
    assert abs(m.max() - linear.spectral_radius(*s, nk=32)) < 1e-12
    assert m.max() > 1.0 + 1e-4 and m[16, 16] == m.max()       # weakly unstable at (pi, pi)
    for name in ("LL", "T5A"):
        assert vn.spectral_radius(rates(name), nk=32) <= 1.0 + 1e-12


def test_batched_screen_equals_the_oracle_per_set():
    rng = np.random.default_rng(5)
    R = np.column_stack([rng.uniform(1.0, 1.9, 12), rng.uniform(1.0, 1.9, 12), rng.uniform(1.0, 1.99, 12),
                         stability.s_from_nu(rng.uniform(1e-4, 1e-2, 12))])
    radius, ok = vn.screen(R, nk=16, chunk=5)
    for i in range(12):
        assert abs(radius[i] - linear.spectral_radius(*R[i], nk=16)) < 1e-12
    assert np.array_equal(ok, radius <= 1.0 + 1e-9)


def test_dispersion_rejects_bad_wavenumbers():
    with pytest.raises(ValueError):
        vn.dispersion(rates("LL"), np.array([0.0, 0.1]))
    with pytest.raises(ValueError):
        vn.dispersion(rates("LL"), np.array([0.2, 0.1]))
