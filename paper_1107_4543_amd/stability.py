"""Linear (von Neumann) stability screen for relaxation sets, used to admit
simulation jobs: a set is admitted when max |eig G(k)| <= 1 + tol on an
nk x nk wavenumber grid (Sec. 4.1; G(k) as in ``vonneumann``)."""
import numpy as np

from . import _lib, vonneumann


def spectral_radius(s_e, s_eps, s_q, s_nu, U=0.0, V=0.0, nk=32):
    return vonneumann.spectral_radius((s_e, s_eps, s_q, s_nu), nk=nk, U=U, V=V)


def s_from_nu(nu):
    """s_nu of a lattice viscosity nu (scalar or array): the library's own
    conversion, lbm_s_from_nu."""
    if np.ndim(nu) == 0:
        return _lib.lbm_s_from_nu(float(nu))
    return np.vectorize(_lib.lbm_s_from_nu, otypes=[np.float64])(np.asarray(nu, dtype=np.float64))


def rates(relax):
    """(s_e, s_eps, s_q, s_nu) of a relaxation dict holding s_nu or nu."""
    s_nu = relax["s_nu"] if "s_nu" in relax else s_from_nu(relax["nu"])
    return relax["s_e"], relax["s_eps"], relax["s_q"], s_nu


def stable(relax, U=0.0, V=0.0, nk=32, tol=1e-9):
    return spectral_radius(*rates(relax), U=U, V=V, nk=nk) <= 1.0 + tol
