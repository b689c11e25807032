"""Linearised (von Neumann) analysis of the D2Q9 MRT scheme, FP64, NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The linear collision operator is the matrix Psi printed in Sec. 2.3 for the
reference state rho0 = 1 with uniform velocity (U, V); it is typed here from
that display and NOT derived from the oracle's nonlinear collision, so that
the two can be checked against each other.  With the linearised step in pull
form (Sec. 2.2, Eq. l-mrt-lbs) a plane wave f'(x) = a exp(i k.x) advances as

    a(t+1) = G(k) a(t),   G(k) = diag(exp(-i k.v_j)) M^{-1} Psi M,

which is the von Neumann matrix of Sec. 4.1 with the undefined matrix "A"
read as diag(exp(i k.v_j)) (the plane-wave shift), so its eigenvalues are
lambda = exp(-i omega).  Hence Re(omega) = -arg(lambda) and
Im(omega) = ln|lambda| per step.
"""
import numpy as np

from . import moment_matrix, velocities, inverse

CS = 1.0 / np.sqrt(3.0)


def sigma_from_s(s):
    """sigma = 1/s - 1/2 (Sec. 2.3)."""
    return 1.0 / np.asarray(s, dtype=np.float64) - 0.5


def s_from_sigma(sigma):
    return 1.0 / (np.asarray(sigma, dtype=np.float64) + 0.5)


def nu_from_s(s_nu):
    """Kinematic shear viscosity nu = sigma_nu / 3 (lattice units); the factor
    1/3 = c_s^2 is read off the first-order dissipation matrix of Sec. 2.3.1
    (shear entries -k^2 sigma_nu / 3) and the Landau-Lifshitz shear mode
    Im(omega^s) = -nu k^2 (Sec. 4.1)."""
    return sigma_from_s(s_nu) / 3.0


def s_from_nu(nu):
    return s_from_sigma(3.0 * np.asarray(nu, dtype=np.float64))


def psi(s_e, s_eps, s_q, s_nu, U=0.0, V=0.0):
    """The 9x9 linear collision matrix Psi at (rho0=1, U, V) as printed in Sec. 2.3."""
    P = np.zeros((9, 9))
    P[0, 0] = P[1, 1] = P[2, 2] = 1.0
    q2 = U * U + V * V
    P[3, 0:3] = [-2.0 * s_e - 3.0 * q2 * s_e, 6.0 * U * s_e, 6.0 * V * s_e]
    P[3, 3] = 1.0 - s_e
    P[4, 0:3] = [s_eps + 3.0 * q2 * s_eps, -6.0 * U * s_eps, -6.0 * V * s_eps]
    P[4, 4] = 1.0 - s_eps
    P[5, 1] = -s_q
    P[5, 5] = 1.0 - s_q
    P[6, 2] = -s_q
    P[6, 6] = 1.0 - s_q
    P[7, 0:3] = [-(U * U - V * V) * s_nu, 2.0 * U * s_nu, -2.0 * V * s_nu]
    P[7, 7] = 1.0 - s_nu
    P[8, 0:3] = [-U * V * s_nu, V * s_nu, U * s_nu]
    P[8, 8] = 1.0 - s_nu
    return P


def collision_matrix(s_e, s_eps, s_q, s_nu, U=0.0, V=0.0):
    """Population-space linear collision M^{-1} Psi M."""
    M = moment_matrix()
    return inverse(M) @ psi(s_e, s_eps, s_q, s_nu, U, V) @ M


def amplification(kx, ky, s_e, s_eps, s_q, s_nu, U=0.0, V=0.0):
    """One-step amplification matrix G(k) acting on the Fourier amplitudes of
    the population fluctuations."""
    cx, cy = velocities()
    shift = np.exp(-1j * (kx * cx + ky * cy))
    return shift[:, None] * collision_matrix(s_e, s_eps, s_q, s_nu, U, V)


def eigen(kx, ky, s_e, s_eps, s_q, s_nu, U=0.0, V=0.0):
    """Eigenvalues and right eigenvectors of G(k)."""
    return np.linalg.eig(amplification(kx, ky, s_e, s_eps, s_q, s_nu, U, V))


def omegas(kx, ky, s_e, s_eps, s_q, s_nu, U=0.0, V=0.0):
    """Complex frequencies omega = i ln(lambda) of all nine modes."""
    lam = np.linalg.eigvals(amplification(kx, ky, s_e, s_eps, s_q, s_nu, U, V))
    return 1j * np.log(lam)


def hydrodynamic_modes(kx, ky, s_e, s_eps, s_q, s_nu, U=0.0, V=0.0):
    """The three eigenvalues of G(k) closest to 1 (two acoustic, one shear),
    with eigenvectors, sorted by the real part of omega (ascending)."""
    lam, vec = eigen(kx, ky, s_e, s_eps, s_q, s_nu, U, V)
    idx = np.argsort(np.abs(lam - 1.0))[:3]
    lam, vec = lam[idx], vec[:, idx]
    om = 1j * np.log(lam)
    order = np.argsort(om.real)
    return lam[order], vec[:, order]


def spectral_radius(s_e, s_eps, s_q, s_nu, U=0.0, V=0.0, nk=64):
    """max |lambda| over an nk x nk grid of wavenumbers in [0, 2 pi)^2."""
    ks = 2.0 * np.pi * np.arange(nk) / nk
    C = collision_matrix(s_e, s_eps, s_q, s_nu, U, V)
    cx, cy = velocities()
    worst = 0.0
    for kx in ks:
        for ky in ks:
            G = np.exp(-1j * (kx * cx + ky * cy))[:, None] * C
            worst = max(worst, float(np.max(np.abs(np.linalg.eigvals(G)))))
    return worst
