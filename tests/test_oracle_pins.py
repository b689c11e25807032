"""Pins of the FP64 oracle's nonlinear step against what the paper and the
mathematics fix (no GPU).

Each test states the passage or textbook fact it checks.  A plausible slip in
the oracle -- a wrong row of M, a wrong sign in the equilibrium, a swapped
relaxation rate, a transposed velocity, a wrong streaming direction -- makes at
least one of them fail.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import linear

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
LL = GOLD["lallemand_luo"]

# Textbook D2Q9 lattice weights (Qian, d'Humieres & Lallemand 1992); used only
# for the independent quadratic equilibrium below.
W_TEXTBOOK = {(0, 0): 4 / 9, (1, 0): 1 / 9, (0, 1): 1 / 9, (-1, 0): 1 / 9, (0, -1): 1 / 9,
              (1, 1): 1 / 36, (-1, 1): 1 / 36, (-1, -1): 1 / 36, (1, -1): 1 / 36}


def feq_textbook(rho, ux, uy):
    cx, cy = oracle.velocities()
    out = []
    for i in range(9):
        w = W_TEXTBOOK[(int(cx[i]), int(cy[i]))]
        cu = cx[i] * ux + cy[i] * uy
        out.append(w * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy)))
    return np.array(out)


def ll_rates(nu=1e-3):
    return [LL["s_e"], LL["s_eps"], LL["s_q"], float(linear.s_from_nu(nu))]


def test_velocity_set_is_d2q9():
    # Sec. 2.1: x + v_j dt must stay on the lattice; D2Q9 = all of {-1,0,1}^2.
    cx, cy = oracle.velocities()
    assert sorted(zip(cx.tolist(), cy.tolist())) == sorted(W_TEXTBOOK)
    assert (cx[0], cy[0]) == (0, 0)


def test_M_rows_orthogonal_with_known_norms():
    # M M^T is diagonal, diag(9,6,6,36,36,12,12,4,4), for the Lallemand-Luo basis.
    M = oracle.moment_matrix()
    G = M @ M.T
    assert np.array_equal(G, np.diag([9.0, 6, 6, 36, 36, 12, 12, 4, 4]))
    # Sec. 2.1: M_0j = 1 and M_alpha j = v_j^alpha.
    cx, cy = oracle.velocities()
    assert np.array_equal(M[0], np.ones(9))
    assert np.array_equal(M[1], cx.astype(float))
    assert np.array_equal(M[2], cy.astype(float))


def test_gauss_jordan_inverse_equals_scaled_transpose():
    # For orthogonal rows, M^{-1} = M^T D^{-1}; the oracle inverts generally.
    M = oracle.moment_matrix()
    Minv = oracle.inverse(M)
    D = np.diag(M @ M.T)
    assert np.max(np.abs(Minv - M.T / D[None, :])) < 1e-15
    assert np.max(np.abs(Minv @ M - np.eye(9))) < 1e-15


@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (1.03, 0.1, -0.05), (0.97, -0.2, 0.15)])
def test_equilibrium_is_textbook_quadratic(rho, ux, uy):
    # Sec. 2.3 gives only m^eq; M^{-1} m^eq must be the standard D2Q9 f^eq.
    f = oracle.init(np.full((1, 1), rho), np.full((1, 1), ux), np.full((1, 1), uy))[:, 0, 0]
    assert np.max(np.abs(f - feq_textbook(rho, ux, uy))) < 2e-16 * 4


def test_equilibrium_moments_printed_form():
    # Sec. 2.3: m^eq = (rho, jx, jy, -2rho+3|j|^2/rho, rho-3|j|^2/rho, -jx, -jy,
    # (jx^2-jy^2)/rho, jx jy/rho) -- checked at a point against M f^eq.
    rho, ux, uy = 1.1, 0.07, -0.03
    M = oracle.moment_matrix()
    m = M @ feq_textbook(rho, ux, uy)
    assert np.max(np.abs(m - oracle.meq(rho, rho * ux, rho * uy))) < 1e-15


def _random_near_eq(rng, n, amp=1e-2):
    rho = 1.0 + amp * rng.standard_normal(n)
    ux = 0.05 * rng.standard_normal(n)
    uy = 0.05 * rng.standard_normal(n)
    f = np.stack([feq_textbook(rho[c], ux[c], uy[c]) for c in range(n)], axis=1)
    return f + amp * 0.1 * rng.standard_normal(f.shape)


def test_collision_conserves_mass_and_momentum_per_cell():
    # Sec. 2.1, Eq. eq_conservative: m_0..m_2 are collision invariants.
    rng = np.random.default_rng(1)
    f = _random_near_eq(rng, 200)
    fs = oracle.collide(f, ll_rates())
    cx, cy = oracle.velocities()
    for w in (np.ones(9), cx.astype(float), cy.astype(float)):
        assert np.max(np.abs(w @ fs - w @ f)) < 8 * 2.2e-16   # a few ulps of rho ~ 1
    # ... and the collision actually changes the non-conserved part.
    assert np.max(np.abs(fs - f)) > 1e-4


def test_equal_rates_reduce_to_bgk():
    # Sec. 2.1, Eq. eq_BGK_LBM_R: Lambda = s I.  With all s_k equal, Lambda =
    # M^{-1} S M acts as s on the non-conserved part, and since f^eq has the
    # same conserved moments as f, f* = f + s (f^eq(rho, u) - f).
    rng = np.random.default_rng(2)
    f = _random_near_eq(rng, 50)
    s = 1.37
    fs = oracle.collide(f, [s, s, s, s])
    cx, cy = oracle.velocities()
    rho = f.sum(0)
    ux = (cx[:, None] * f).sum(0) / rho
    uy = (cy[:, None] * f).sum(0) / rho
    fe = np.stack([feq_textbook(rho[c], ux[c], uy[c]) for c in range(f.shape[1])], axis=1)
    assert np.max(np.abs(fs - (f + s * (fe - f)))) < 1e-15


@pytest.mark.parametrize("U,V", [(0.0, 0.0), (0.1, 0.03), (-0.05, 0.12)])
def test_collision_jacobian_is_printed_psi(U, V):
    # Sec. 2.3: the collision linearised at (rho0=1, U, V) in moment space is
    # the printed matrix Psi.  Central differences of the oracle's nonlinear
    # collision, mapped to moment space, must reproduce it.
    s = [1.64, 1.54, 1.9, 1.2]
    M = oracle.moment_matrix()
    Minv = oracle.inverse(M)
    f0 = feq_textbook(1.0, U, V)
    h = 1e-6
    J = np.zeros((9, 9))
    for j in range(9):
        dm = np.zeros(9)
        dm[j] = h
        fp = oracle.collide((f0 + Minv @ dm)[:, None], s)[:, 0]
        fm = oracle.collide((f0 - Minv @ dm)[:, None], s)[:, 0]
        J[:, j] = M @ (fp - fm) / (2 * h)
    P = linear.psi(*s, U=U, V=V)
    assert np.max(np.abs(J - P)) < 1e-8


def test_uniform_equilibrium_is_a_fixed_point():
    rho = np.full((5, 7), 1.0)
    ux = np.full((5, 7), 0.0577)
    uy = np.full((5, 7), -0.02)
    f0 = oracle.init(rho, ux, uy)
    f = oracle.run(f0, ll_rates(), 20)
    assert np.max(np.abs(f - f0)) < 1e-15


def test_stream_moves_each_population_along_its_velocity():
    # Sec. 2.1, Eq. blbs: f_i(x + v_i, t + 1) = f*_i(x); periodic wrap.
    nx, ny = 5, 4
    cx, cy = oracle.velocities()
    for (x0, y0) in [(2, 1), (0, 0), (4, 3), (0, 3)]:
        fs = np.zeros((9, ny, nx))
        for i in range(9):
            fs[i, y0, x0] = 1.0 + i
        f = oracle.stream(fs)
        for i in range(9):
            xd, yd = (x0 + cx[i]) % nx, (y0 + cy[i]) % ny
            assert f[i, yd, xd] == 1.0 + i
            assert np.count_nonzero(f[i]) == 1


def test_translation_invariance_is_bitwise():
    rng = np.random.default_rng(3)
    ny, nx = 12, 16
    rho = 1 + 1e-3 * rng.standard_normal((ny, nx))
    ux = 1e-3 * rng.standard_normal((ny, nx))
    uy = 1e-3 * rng.standard_normal((ny, nx))
    f0 = oracle.init(rho, ux, uy)
    a = oracle.run(f0, ll_rates(), 7)
    b = oracle.run(np.roll(f0, (3, -5), axis=(1, 2)), ll_rates(), 7)
    assert np.array_equal(np.roll(a, (3, -5), axis=(1, 2)), b)


def test_y_uniform_field_stays_bitwise_y_uniform_and_equals_one_row():
    import lbm_inputs
    s = [1.99, 1.962820428, 1.992761413, 1.999960001]
    rho, ux, uy = lbm_inputs.plane_waves(64, 8, 2, 1e-4, 1e-4, 0.1 * lbm_inputs.CS)
    f = oracle.run(oracle.init(rho, ux, uy), s, 30)
    assert all(np.array_equal(f[:, 0], f[:, y]) for y in range(8))
    f1 = oracle.run(oracle.init(rho[:1], ux[:1], uy[:1]), s, 30)
    assert np.array_equal(f1[:, 0], f[:, 0])


def test_centred_pulse_symmetry():
    import lbm_inputs
    n = 32
    rho, ux, uy = lbm_inputs.gaussian_pulse(n, n, 1e-3, 4.0)
    f = oracle.run(oracle.init(rho, ux, uy), ll_rates(), 40)
    r, _, _ = oracle.moments(f)
    c = n // 2
    idx = (np.arange(n) * -1 + 2 * c) % n          # x -> 2c - x
    assert np.max(np.abs(r - r[:, idx])) < 1e-14
    assert np.max(np.abs(r - r[idx, :])) < 1e-14
    assert np.max(np.abs(r - r.T)) < 1e-14


def test_global_conservation_over_a_run():
    import lbm_inputs
    rho, ux, uy = lbm_inputs.gaussian_pulse(48, 40, 1e-3, 4.0, u0=(0.05, 0.0))
    f0 = oracle.init(rho, ux, uy)
    f = oracle.run(f0, ll_rates(), 100)
    cx, cy = oracle.velocities()
    for w in (np.ones(9), cx.astype(float), cy.astype(float)):
        a = np.einsum("i,iyx->", w, f0)
        b = np.einsum("i,iyx->", w, f)
        assert abs(a - b) < 1e-11


@pytest.mark.parametrize("mx,my,U,V", [(3, 0, 0.0, 0.0), (2, 5, 0.0, 0.0), (4, 1, 0.08, -0.03),
                                       (9, 9, 0.0, 0.0)])
def test_one_step_small_plane_wave_matches_linear_amplification(mx, my, U, V):
    # Sec. 4.1: a small fluctuation f' = Re(a e^{ik.x}) about the uniform state
    # (rho0 = 1, U, V) advances by G(k) = diag(e^{-ik.v}) M^{-1} Psi M.  The
    # oracle's nonlinear step must match it to O(amplitude).
    nx, ny = 24, 20
    s = [1.64, 1.54, 1.9, 1.7]
    kx, ky = 2 * np.pi * mx / nx, 2 * np.pi * my / ny
    rng = np.random.default_rng(mx * 31 + my)
    a = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    eps = 1e-7
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    phase = np.exp(1j * (kx * X + ky * Y))
    base = feq_textbook(1.0, U, V)[:, None, None]
    f0 = base + eps * np.real(a[:, None, None] * phase[None])
    f1 = oracle.run(f0, s, 1)
    proj = ((f1 - base) * np.conj(phase)[None]).sum(axis=(1, 2)) * 2 / (nx * ny) / eps
    if (2 * mx) % nx == 0 and (2 * my) % ny == 0:
        pytest.skip("self-conjugate mode")
    pred = linear.amplification(kx, ky, *s, U=U, V=V) @ a
    assert np.max(np.abs(proj - pred)) < 1e-6 * np.max(np.abs(a))


def test_s_nu_from_viscosity_matches_table4():
    # Table 4 prints nu next to s_nu; nu = (1/s_nu - 1/2)/3 must reproduce it.
    for g in ("A", "B"):
        row = GOLD["table4"][g]
        assert abs(float(linear.nu_from_s(row["s_nu"])) - row["nu"]) < 6e-9


def test_table3_sigma_form_equals_table5_rates():
    # Sec. 2.3: sigma = 1/s - 1/2; Table 3 (sigma) and Table 5 (s) print the
    # same optimised sets.
    for g in ("A", "B"):
        t3, t5 = GOLD["table3"][g], GOLD["table5"][g]
        for k in ("e", "nu", "eps", "q"):
            s = float(linear.s_from_sigma(t3["sigma_" + k]))
            assert abs(s - t5["s_" + k]) < 1e-8, (g, k)


def test_window_run_reproduces_the_centre_of_a_larger_periodic_run():
    # A cell's value after T steps depends only on cells within distance T,
    # so an oracle run on a periodic window of side 2T + 1 + 2r reproduces the
    # central (2r + 1)^2 block of the run on the whole lattice exactly (the
    # basis of the sampled full-size parity checks).
    import lbm_inputs
    nx = ny = 64
    T, r = 9, 2
    specs = lbm_inputs.random_pulse_specs(nx, ny, seed=5, count=6, width_range=(2.0, 5.0))
    full = oracle.run(oracle.init(*lbm_inputs.pulses_field(nx, ny, specs)), ll_rates(), T)
    w = 2 * T + 1 + 2 * r
    x0, y0 = 50, 3                                   # window wraps around the lattice edge
    win = oracle.run(oracle.init(*lbm_inputs.pulses_window(nx, ny, specs, x0, y0, w)), ll_rates(), T)
    c = slice(T, T + 2 * r + 1)
    ys = (y0 + np.arange(w))[c] % ny
    xs = (x0 + np.arange(w))[c] % nx
    assert np.array_equal(win[:, c, c], full[:, ys][:, :, xs])
    # a window two cells too small (side 2T - 1) around the same centre cell
    # lets wrapped values reach it, and the centre then differs
    gx, gy = (x0 + T + r) % nx, (y0 + T + r) % ny
    small = oracle.run(oracle.init(*lbm_inputs.pulses_window(nx, ny, specs, gx - (T - 1), gy - (T - 1),
                                                              2 * T - 1)), ll_rates(), T)
    assert np.array_equal(win[:, T + r, T + r], full[:, gy, gx])
    assert not np.array_equal(small[:, T - 1, T - 1], full[:, gy, gx])


def test_unstable_relaxation_set_blows_up_in_the_oracle():
    # A set outside the von Neumann stability region (max |lambda| = 1.14 at
    # the checkerboard mode) must blow up; the linear analysis predicts it.
    import lbm_inputs
    s = [1.860, 1.075, 1.312, 1.9169]
    assert linear.spectral_radius(*s, nk=16) > 1.1
    rho, ux, uy = lbm_inputs.gaussian_pulse(64, 64, 1e-3, 4.0)
    f = oracle.run(oracle.init(rho, ux, uy), s, 600)
    assert not np.all(np.isfinite(f)) or np.max(np.abs(f)) > 1e3


def test_moments_of_single_population_cells():
    # Sec. 2.1, Eq. q-macro: rho = sum_i f_i and rho u = sum_i v_i f_i.  A cell
    # holding mass a in population i alone has density a and moves with that
    # population's lattice velocity v_i exactly: a missing 1/rho (a != 1), a
    # swapped or mis-signed velocity component, or a population left out of a
    # sum fails here.
    cx, cy = oracle.velocities()
    a = np.array([0.5, 1.0, 2.0, 3.25])
    for i in range(9):
        f = np.zeros((9, 1, a.size))
        f[i, 0, :] = a
        rho, ux, uy = oracle.moments(f)
        assert np.array_equal(rho[0], a)
        assert np.array_equal(ux[0], np.full(a.size, float(cx[i])))
        assert np.array_equal(uy[0], np.full(a.size, float(cy[i])))


def test_moments_of_two_population_cell_weigh_by_mass():
    # Two populations: rho u = a v_i + b v_j, divided by rho = a + b.
    cx, cy = oracle.velocities()
    f = np.zeros((9, 1, 1))
    f[1, 0, 0], f[6, 0, 0] = 3.0, 1.0          # (1,0) with mass 3, (-1,1) with mass 1
    rho, ux, uy = oracle.moments(f)
    jx = 3.0 * cx[1] + 1.0 * cx[6]
    jy = 3.0 * cy[1] + 1.0 * cy[6]
    assert (jx, jy) == (2, 1)                   # the D2Q9 directions of those populations
    assert rho[0, 0] == 4.0 and ux[0, 0] == 0.5 and uy[0, 0] == 0.25


def test_moments_of_textbook_equilibrium_are_its_density_and_velocity():
    # The textbook quadratic f^eq (Qian et al.) has zeroth moment rho and first
    # moment rho u exactly (closed-form lattice sums), so the readback of
    # random equilibrium fields must return those fields to a few ulps.
    rng = np.random.default_rng(7)
    ny, nx = 5, 6
    rho = 1.0 + 0.2 * rng.standard_normal((ny, nx))
    ux = 0.1 * rng.standard_normal((ny, nx))
    uy = 0.1 * rng.standard_normal((ny, nx))
    f = np.stack([feq_textbook(rho, ux, uy)[i] for i in range(9)])
    r, u, v = oracle.moments(f)
    assert np.max(np.abs(r - rho)) < 8e-16
    assert np.max(np.abs(u - ux)) < 8e-16
    assert np.max(np.abs(v - uy)) < 8e-16
    # and the same through the oracle's own initialisation
    r2, u2, v2 = oracle.moments(oracle.init(rho, ux, uy))
    assert np.max(np.abs(r2 - rho)) < 8e-16
    assert np.max(np.abs(u2 - ux)) < 8e-16 and np.max(np.abs(v2 - uy)) < 8e-16
