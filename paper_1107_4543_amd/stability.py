"""Linear (von Neumann) stability screen for relaxation sets, used to admit
simulation jobs.  Host logic, NumPy.

The linearised collision about the uniform state (rho0 = 1, U, V) maps the
moment fluctuation m' to (I - S (I - dmeq/dm)) m', with dmeq/dm the Jacobian
of the D2Q9 equilibrium moments (Sec. 2.3) at that state; one step of a plane
wave exp(i k.x) multiplies the population amplitudes by
G(k) = diag(exp(-i k.v)) M^{-1} (I - S (I - dmeq/dm)) M.  A relaxation set is
admitted when max |eig G(k)| <= 1 + tol on an nk x nk wavenumber grid.
"""
import numpy as np

_CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
_CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)


def _moment_matrix():
    c2 = _CX ** 2 + _CY ** 2
    return np.stack([np.ones(9), _CX, _CY, 3 * c2 - 4, 4.5 * c2 ** 2 - 10.5 * c2 + 4,
                     (3 * c2 - 5) * _CX, (3 * c2 - 5) * _CY, _CX ** 2 - _CY ** 2, _CX * _CY])


def _equilibrium_jacobian(U, V):
    """d m^eq / d (rho, jx, jy) at rho = 1, j = (U, V), padded to 9 x 9."""
    J = np.zeros((9, 9))
    J[0, 0] = J[1, 1] = J[2, 2] = 1.0
    q = U * U + V * V
    J[3, :3] = [-2.0 - 3.0 * q, 6.0 * U, 6.0 * V]
    J[4, :3] = [1.0 + 3.0 * q, -6.0 * U, -6.0 * V]
    J[5, 1] = -1.0
    J[6, 2] = -1.0
    J[7, :3] = [-(U * U - V * V), 2.0 * U, -2.0 * V]
    J[8, :3] = [-U * V, V, U]
    return J


def spectral_radius(s_e, s_eps, s_q, s_nu, U=0.0, V=0.0, nk=32):
    M = _moment_matrix()
    S = np.diag([0.0, 0.0, 0.0, s_e, s_eps, s_q, s_q, s_nu, s_nu])
    C = np.linalg.solve(M, (np.eye(9) - S @ (np.eye(9) - _equilibrium_jacobian(U, V))) @ M)
    k = 2.0 * np.pi * np.arange(nk) / nk
    KX, KY = np.meshgrid(k, k, indexing="ij")
    phase = np.exp(-1j * (KX[..., None] * _CX + KY[..., None] * _CY))        # [nk, nk, 9]
    G = phase[..., :, None] * C[None, None]
    return float(np.max(np.abs(np.linalg.eigvals(G.reshape(-1, 9, 9)))))


def s_from_nu(nu):
    return 1.0 / (3.0 * nu + 0.5)


def rates(relax):
    """(s_e, s_eps, s_q, s_nu) of a relaxation dict holding s_nu or nu."""
    s_nu = relax["s_nu"] if "s_nu" in relax else s_from_nu(relax["nu"])
    return relax["s_e"], relax["s_eps"], relax["s_q"], s_nu


def stable(relax, U=0.0, V=0.0, nk=32, tol=1e-9):
    return spectral_radius(*rates(relax), U=U, V=V, nk=nk) <= 1.0 + tol
