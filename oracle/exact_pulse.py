"""Exact density of the acoustic Gaussian pressure pulse (Sec. 5.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For the initial condition rho = rho0 + eps exp(-alpha eta^2), u = (U0, 0),
alpha = ln 2 / b^2, the linear inviscid solution is

    rho(x, y, t) = rho0 + eps / (2 alpha) * int_0^inf exp(-xi^2 / (4 alpha))
                          cos(c_s xi t) J0(xi eta) xi dxi,
    eta = sqrt((x - U0 t)^2 + y^2),

the zero-order Hankel transform of the Gaussian propagated with the sound
speed c_s.  Everything here is in lattice units (cells, steps, c_s = 1/sqrt 3).

The integral is evaluated by Gauss-Legendre quadrature on [0, xi_max], where
exp(-xi_max^2 / (4 alpha)) = e^-46 (below FP64 resolution relative to the
peak); the integrand oscillates about 2 (c_s t + eta) xi_max / (2 pi) times,
and the node count is chosen to resolve that with a wide margin.
"""
import math

import numpy as np
from scipy.special import j0

CS = 1.0 / math.sqrt(3.0)


def _nodes(alpha, reach):
    xi_max = math.sqrt(4.0 * alpha * 46.0)
    oscillations = reach * xi_max / (2.0 * math.pi)
    n = int(max(200, 40 * oscillations + 100))
    x, w = np.polynomial.legendre.leggauss(n)
    xi = 0.5 * xi_max * (x + 1.0)
    return xi, 0.5 * xi_max * w


def density(eta, t, amplitude, half_width, rho0=1.0, cs=CS, chunk=4096):
    """rho at radial distance(s) eta (array) from the advected pulse centre at time t."""
    eta = np.asarray(eta, dtype=np.float64)
    alpha = math.log(2.0) / half_width ** 2
    xi, w = _nodes(alpha, cs * t + float(np.max(eta, initial=0.0)))
    kern = w * np.exp(-xi * xi / (4.0 * alpha)) * np.cos(cs * xi * t) * xi
    flat = eta.ravel()
    out = np.empty_like(flat)
    for s in range(0, flat.size, chunk):
        e = flat[s:s + chunk]
        out[s:s + chunk] = j0(np.outer(e, xi)) @ kern
    return rho0 + amplitude / (2.0 * alpha) * out.reshape(eta.shape)


def field(nx, ny, t, amplitude, half_width, center, u0x=0.0, rho0=1.0):
    """Exact rho on an nx x ny grid (cell centres at integer coordinates) with
    the pulse started at `center` and advected by u0x; distances are taken as
    the minimum image on the periodic lattice."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    dx = x - (center[0] + u0x * t)
    dx = dx - nx * np.round(dx / nx)
    dy = y - center[1]
    dy = dy - ny * np.round(dy / ny)
    eta = np.sqrt(dx * dx + dy * dy)
    return density(eta, t, amplitude, half_width, rho0)
