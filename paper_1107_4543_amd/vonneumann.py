"""Von Neumann (linear) analysis of the D2Q9 MRT scheme (Sec. 4.1).

A small plane-wave perturbation f' = a exp(i k.x) of the uniform state
(rho0 = 1, U, V) is multiplied per step by

    G(k) = diag(exp(-i k.v)) M^{-1} (I - S (I - J)) M,

with M the moment matrix, S the relaxation rates and J the Jacobian of the
equilibrium moments m^eq(rho, j) (Sec. 2.3) at that state.  An eigenvalue
lambda of G defines the complex frequency omega = i ln(lambda): the mode
advances its phase by Re(omega) per step (phase speed Re(omega)/|k|) and
grows by Im(omega) (dissipation -Im(omega)).  Three eigenvalues tend to 1 as
k -> 0: two acoustic modes and one shear mode; the other six are kinetic
modes that relax at rates set by the non-conserved s_k.

Everything here is host analysis in FP64 (NumPy), batched over arrays of
wavenumbers, mean flows and relaxation sets:

* ``amplification`` / ``spectrum``   G(k) and its eigen-decomposition;
* ``dispersion``                     the nine modes tracked along |k| in one
                                     direction, the three hydrodynamic ones
                                     labelled, with phase speed and
                                     dissipation curves;
* ``navier_stokes``                  the linearised isothermal
                                     Navier-Stokes modes the scheme is meant
                                     to reproduce;
* ``stability_map`` / ``screen``     max |lambda| over the wavenumber plane,
                                     for one relaxation set or many;
* ``measure_dispersion``             the same frequencies measured on the
                                     GPU: small plane waves are stepped by
                                     the library's kernels and projected
                                     every step (``lbm_project``), and each
                                     eigen-coordinate is fitted.
"""
import math
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np
from scipy.optimize import linear_sum_assignment

CS = 1.0 / math.sqrt(3.0)
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
NORMS = np.array([9.0, 6.0, 6.0, 36.0, 36.0, 12.0, 12.0, 4.0, 4.0])
HYDRO = ("acoustic-", "shear", "acoustic+")


def moment_matrix():
    c2 = CX ** 2 + CY ** 2
    return np.stack([np.ones(9), CX, CY, 3 * c2 - 4, 4.5 * c2 ** 2 - 10.5 * c2 + 4,
                     (3 * c2 - 5) * CX, (3 * c2 - 5) * CY, CX ** 2 - CY ** 2, CX * CY])


_M = moment_matrix()
_MINV = _M.T / NORMS            # the rows of M are orthogonal with squared norms NORMS


def _rate_diagonal(rates):
    r = np.asarray(rates, dtype=np.float64)
    s_e, s_eps, s_q, s_nu = (r[..., i] for i in range(4))
    z = np.zeros_like(s_e)
    return np.stack([z, z, z, s_e, s_eps, s_q, s_q, s_nu, s_nu], axis=-1)


def equilibrium_jacobian(U, V):
    """d m^eq / d(rho, jx, jy) at rho = 1, j = (U, V), as 9 x 9 (zero columns
    for the non-conserved moments); broadcasts over U, V."""
    U, V = np.broadcast_arrays(np.asarray(U, dtype=np.float64), np.asarray(V, dtype=np.float64))
    J = np.zeros(U.shape + (9, 9))
    J[..., 0, 0] = J[..., 1, 1] = J[..., 2, 2] = 1.0
    q = U * U + V * V
    J[..., 3, 0], J[..., 3, 1], J[..., 3, 2] = -2.0 - 3.0 * q, 6.0 * U, 6.0 * V
    J[..., 4, 0], J[..., 4, 1], J[..., 4, 2] = 1.0 + 3.0 * q, -6.0 * U, -6.0 * V
    J[..., 5, 1] = -1.0
    J[..., 6, 2] = -1.0
    J[..., 7, 0], J[..., 7, 1], J[..., 7, 2] = -(U * U - V * V), 2.0 * U, -2.0 * V
    J[..., 8, 0], J[..., 8, 1], J[..., 8, 2] = -U * V, V, U
    return J


def collision_operator(rates, U=0.0, V=0.0):
    """Linearised collision in population space, M^{-1}(I - S(I - J))M;
    rates is (s_e, s_eps, s_q, s_nu) or an array [..., 4]."""
    S = _rate_diagonal(rates)
    J = equilibrium_jacobian(U, V)
    S, J = np.broadcast_arrays(S[..., :, None], J)
    A = np.eye(9) - S * (np.eye(9) - J)
    return _MINV @ A @ _M


def amplification(rates, kx, ky, U=0.0, V=0.0):
    """G(k), broadcast over rates [..., 4], kx, ky, U and V."""
    C = collision_operator(rates, U, V)
    kx, ky = np.asarray(kx, dtype=np.float64), np.asarray(ky, dtype=np.float64)
    phase = np.exp(-1j * (kx[..., None] * CX + ky[..., None] * CY))
    shape = np.broadcast_shapes(phase.shape[:-1], C.shape[:-2])
    return np.broadcast_to(phase, shape + (9,))[..., :, None] * np.broadcast_to(C, shape + (9, 9))


def spectrum(rates, kx, ky, U=0.0, V=0.0):
    """Eigenvalues [..., 9] and right eigenvectors [..., 9, 9] of G(k)."""
    return np.linalg.eig(amplification(rates, kx, ky, U, V))


def omega(lam):
    """Complex frequency i ln(lambda): Re = phase per step, Im = growth per step."""
    return 1j * np.log(lam)


def conserved_weight(vec):
    """Share of each eigenvector's (D-normalised) moment content carried by
    the conserved moments rho, jx, jy; vec is [..., 9, n] (columns)."""
    m = np.einsum("ij,...jn->...in", _M, vec)
    w = np.abs(m) ** 2 / NORMS[:, None]
    return w[..., :3, :].sum(axis=-2) / w.sum(axis=-2)


@dataclass
class Dispersion:
    k: np.ndarray            # [n] wavenumber magnitudes
    theta: float
    lam: np.ndarray          # [n, 9] eigenvalues, columns tracked along k
    vec: np.ndarray          # [n, 9, 9]
    labels: List[str]        # per column: acoustic-, shear, acoustic+ or kinetic

    @property
    def omega(self):
        """[n, 9]; Re(omega) continuous along k."""
        om = omega(self.lam)
        return np.unwrap(om.real, axis=0) + 1j * om.imag

    def column(self, label):
        return self.labels.index(label)

    def phase_speed(self, label):
        return self.omega[:, self.column(label)].real / self.k

    def dissipation(self, label):
        return -self.omega[:, self.column(label)].imag


def dispersion(rates, k, theta=0.0, U=0.0, V=0.0):
    """The nine modes along k (ascending, k[0] small enough that the three
    hydrodynamic modes are the ones carried by the conserved moments) in
    direction theta.  Columns are tracked from one k to the next by maximal
    eigenvector overlap; the hydrodynamic columns are labelled at k[0] by
    their phase speed relative to the mean flow."""
    k = np.asarray(k, dtype=np.float64)
    if k.ndim != 1 or k.size < 1 or np.any(np.diff(k) <= 0) or k[0] <= 0:
        raise ValueError("k must be a strictly increasing array of positive wavenumbers")
    lam, vec = spectrum(rates, k * math.cos(theta), k * math.sin(theta), U, V)
    lam, vec = lam.copy(), vec.copy()
    for n in range(1, k.size):
        a = vec[n - 1] / np.linalg.norm(vec[n - 1], axis=0)
        b = vec[n] / np.linalg.norm(vec[n], axis=0)
        overlap = np.abs(a.conj().T @ b)                    # [prev column, new column]
        _, cols = linear_sum_assignment(-overlap)
        lam[n], vec[n] = lam[n][cols], vec[n][:, cols]
    w = conserved_weight(vec[0])
    hyd = np.argsort(w)[-3:]
    speed = -np.angle(lam[0][hyd]) / k[0]
    labels = ["kinetic"] * 9
    for name, j in zip(HYDRO, hyd[np.argsort(speed)]):
        labels[j] = name
    return Dispersion(k, float(theta), lam, vec, labels)


def navier_stokes(k, theta, rates, U=0.0, V=0.0):
    """Linearised isothermal Navier-Stokes frequencies for the viscosities
    the rates imply (nu = (1/s_nu - 1/2)/3, bulk (1/s_e - 1/2)/3): a dict
    label -> omega [n], acoustic Re = k(U.khat +- c_s), Im = -(nu + bulk)/2 k^2,
    shear Re = k U.khat, Im = -nu k^2."""
    s_e, _, _, s_nu = (float(x) for x in rates)
    nu, bulk = (1.0 / s_nu - 0.5) / 3.0, (1.0 / s_e - 0.5) / 3.0
    k = np.asarray(k, dtype=np.float64)
    adv = U * math.cos(theta) + V * math.sin(theta)
    return {"acoustic+": k * (adv + CS) - 0.5j * (nu + bulk) * k * k,
            "acoustic-": k * (adv - CS) - 0.5j * (nu + bulk) * k * k,
            "shear": k * adv - 1j * nu * k * k}


def _k_grid(nk):
    ks = 2.0 * np.pi * np.arange(nk) / nk
    return np.meshgrid(ks, ks, indexing="ij")


def stability_map(rates, nk=64, U=0.0, V=0.0):
    """max |lambda| at each point of the nk x nk wavenumber grid over
    [0, 2 pi)^2 (rows kx, columns ky)."""
    KX, KY = _k_grid(nk)
    return np.abs(np.linalg.eigvals(amplification(rates, KX, KY, U, V))).max(axis=-1)


def spectral_radius(rates, nk=64, U=0.0, V=0.0):
    return float(stability_map(rates, nk, U, V).max())


def screen(rate_sets, nk=32, U=0.0, V=0.0, tol=1e-9, chunk=64):
    """Spectral radius of each relaxation set in rate_sets [n, 4] and whether
    it is at most 1 + tol (linearly stable on the grid)."""
    R = np.asarray(rate_sets, dtype=np.float64).reshape(-1, 4)
    KX, KY = _k_grid(nk)
    radius = np.empty(len(R))
    for i in range(0, len(R), chunk):
        G = amplification(R[i:i + chunk, None, None, :], KX, KY, U, V)
        radius[i:i + chunk] = np.abs(np.linalg.eigvals(G)).max(axis=(-1, -2, -3))
    return radius, radius <= 1.0 + tol


@dataclass
class MeasuredWave:
    wave: tuple              # lattice mode (mx, my)
    kx: float
    ky: float
    lam: np.ndarray          # [9] predicted eigenvalues of G(k)
    conserved: np.ndarray    # [9] conserved-moment share of each eigenvector
    omega: np.ndarray        # [9] measured omega, nan where the mode was not fitted
    points: np.ndarray       # [9] steps used in each fit


def measure_dispersion(rates, waves: Sequence[tuple], nx, ny, steps, U=0.0, V=0.0, storage="f64",
                       amplitude=1e-6, device="cuda:0", floor=1e-6, min_points=16):
    """Steps a superposition of small plane waves (one per lattice mode
    (mx, my) in waves: density A cos(k.x) and transverse velocity
    A sin(k.x)) with the library's kernels, projects the population
    fluctuation on every mode after every step (FP64, on the device), and
    fits each eigen-coordinate of G(k) with an excited amplitude over the
    steps where it stays above floor times its start: lambda by one-step
    least squares, sum c(t+1) conj(c(t)) / sum |c(t)|^2, and omega = i ln lambda."""
    import torch
    from .lattice import Lattice

    waves = [tuple(int(m) for m in w) for w in waves]
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    rho = np.ones((ny, nx))
    ux = np.full((ny, nx), float(U))
    uy = np.full((ny, nx), float(V))
    ks = []
    for mx, my in waves:
        kx, ky = 2.0 * np.pi * mx / nx, 2.0 * np.pi * my / ny
        kn = math.hypot(kx, ky)
        if kn == 0.0:
            raise ValueError("mode (0, 0) carries no wave")
        ph = kx * x + ky * y
        rho += amplitude * np.cos(ph)
        ux += amplitude * np.sin(ph) * (-ky / kn)
        uy += amplitude * np.sin(ph) * (kx / kn)
        ks.append((kx, ky))
    lat = Lattice(nx, ny, *rates, storage=storage, u0=(U, V), device=device)
    lat.init(rho, ux, uy)
    proj = torch.empty((steps + 1, len(waves), 18), dtype=torch.float64, device=device)
    for t in range(steps + 1):
        for w, (mx, my) in enumerate(waves):
            lat.project(mx, my, out=proj[t, w])
        if t < steps:
            lat.step(1)
    P = proj.cpu().numpy()
    lat.close()
    out = []
    for w, (kx, ky) in enumerate(ks):
        a = P[:, w, 0::2] + 1j * P[:, w, 1::2]                 # [t, 9]
        lam, vec = spectrum(rates, kx, ky, U, V)
        c = a @ np.linalg.inv(vec).T                           # eigen-coordinates
        amp = np.abs(c)
        top = amp[0].max()
        om = np.full(9, np.nan + 0j)
        npts = np.zeros(9, dtype=np.int64)
        for j in range(9):
            if amp[0, j] < 1e-3 * top:
                continue
            alive = amp[:, j] > floor * amp[0, j]
            n = int(np.argmin(alive)) if not alive.all() else steps + 1
            if n < min_points:
                continue
            # one-step least squares: exact for c(t) = c0 lambda^t, and free
            # of the phase-unwrapping ambiguity when lambda is near -1
            lam_fit = np.vdot(c[:n - 1, j], c[1:n, j]) / np.vdot(c[:n - 1, j], c[:n - 1, j])
            om[j] = omega(lam_fit)
            npts[j] = n
        out.append(MeasuredWave(waves[w], kx, ky, lam, conserved_weight(vec), om, npts))
    return out
