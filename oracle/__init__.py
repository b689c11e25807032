"""FP64 CPU oracle for the D2Q9 MRT lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares
no code with the GPU path.

* ``oracle.init / collide / stream / run / moments`` wrap the plain C
  implementation in ``lbm_oracle.c`` (absolute variables, unfused two-pass
  collide-then-stream, Sec. 2.1 and Sec. 2.3 of the paper).
* ``oracle.linear`` holds the linearised (von Neumann) analysis built from
  the paper's printed linear collision matrix Psi (Sec. 2.3, Sec. 4.1).
* ``oracle.exact_pulse`` evaluates the exact acoustic pulse solution
  (Sec. 5.2).
* ``oracle.storage`` is the rounding twin for 16-bit population storage.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbm_oracle.so")
_lib = None

Q = 9


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_velocities.argtypes = [ip, ip]
    lib.oracle_velocities.restype = None
    lib.oracle_build_M.argtypes = [dp]
    lib.oracle_build_M.restype = None
    lib.oracle_invert.argtypes = [dp, dp, ctypes.c_int]
    lib.oracle_invert.restype = ctypes.c_int
    lib.oracle_meq.argtypes = [ctypes.c_double] * 3 + [dp]
    lib.oracle_meq.restype = None
    lib.oracle_init.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp, dp, dp]
    lib.oracle_init.restype = ctypes.c_int
    lib.oracle_collide.argtypes = [ctypes.c_int64, dp, dp, dp]
    lib.oracle_collide.restype = ctypes.c_int
    lib.oracle_stream.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp]
    lib.oracle_stream.restype = None
    lib.oracle_run.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp, ctypes.c_int64, dp]
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_moments.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp, dp, dp]
    lib.oracle_moments.restype = None
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    _lib = lib
    return lib


def _p(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _rates(s):
    s = np.ascontiguousarray(np.asarray(s, dtype=np.float64).reshape(4))
    return s


def velocities():
    """(cx, cy) integer arrays of the D2Q9 velocity set in the oracle's order."""
    cx = np.zeros(Q, np.int32)
    cy = np.zeros(Q, np.int32)
    _load().oracle_velocities(cx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              cy.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return cx, cy


def moment_matrix():
    """The 9x9 transformation matrix M (rows: rho, jx, jy, e, eps, qx, qy, pxx, pxy)."""
    M = np.zeros((Q, Q))
    _load().oracle_build_M(_p(M))
    return M


def inverse(A):
    """Gauss-Jordan inverse of a square matrix of order <= 9."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    out = np.zeros_like(A)
    if _load().oracle_invert(_p(A), _p(out), A.shape[0]) != 0:
        raise np.linalg.LinAlgError("singular matrix")
    return out


def meq(rho, jx, jy):
    """Equilibrium moment vector m^eq(rho, jx, jy) (Sec. 2.3)."""
    out = np.zeros(Q)
    _load().oracle_meq(float(rho), float(jx), float(jy), _p(out))
    return out


def init(rho, ux, uy):
    """Equilibrium populations f = M^{-1} m^eq(rho, rho u); returns [9, ny, nx]."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    ux = np.ascontiguousarray(ux, dtype=np.float64)
    uy = np.ascontiguousarray(uy, dtype=np.float64)
    ny, nx = rho.shape
    f = np.zeros((Q, ny, nx))
    if _load().oracle_init(nx, ny, _p(rho), _p(ux), _p(uy), _p(f)) != 0:
        raise RuntimeError("oracle_init failed")
    return f


def collide(f, s):
    """Post-collision populations of independent cells; f is [9, ...]."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    n = f.size // Q
    out = np.zeros_like(f)
    if _load().oracle_collide(n, _p(_rates(s)), _p(f), _p(out)) != 0:
        raise RuntimeError("oracle_collide failed")
    return out


def stream(fstar):
    """Periodic streaming of post-collision populations [9, ny, nx]."""
    fstar = np.ascontiguousarray(fstar, dtype=np.float64)
    _, ny, nx = fstar.shape
    out = np.zeros_like(fstar)
    _load().oracle_stream(nx, ny, _p(fstar), _p(out))
    return out


def run(f, s, nsteps):
    """Returns the pre-collision state after nsteps steps of collide + stream."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _, ny, nx = f.shape
    work = np.zeros_like(f)
    if _load().oracle_run(nx, ny, _p(_rates(s)), _p(f), int(nsteps), _p(work)) != 0:
        raise RuntimeError("oracle_run failed")
    return f


def moments(f):
    """(rho, ux, uy) fields of populations f [9, ny, nx]."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    rho = np.zeros((ny, nx))
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    _load().oracle_moments(nx, ny, _p(f), _p(rho), _p(ux), _p(uy))
    return rho, ux, uy


def threads():
    return int(_load().oracle_threads())


def set_threads(n):
    """Number of OpenMP threads for later calls (results do not depend on it)."""
    _load().oracle_set_threads(int(n))
