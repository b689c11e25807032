"""ctypes binding of the C ABI declared in include/lbm.h (argument marshalling
only).  Every function keeps its C name; failures raise ``LbmError`` carrying
the status code and the library's message.  The library must have been built
(``python paper_1107_4543_amd/build.py``); there is no fallback."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK = 0
LBM_E_INVAL = -1
LBM_E_NOMEM = -2
LBM_E_HIP = -3
LBM_E_NONFINITE = -4
LBM_E_STATE = -5

LBM_STORE_F64, LBM_STORE_F32, LBM_STORE_F16, LBM_STORE_BF16 = 0, 1, 2, 3
LBM_COMPUTE_F64, LBM_COMPUTE_F32 = 0, 1
LBM_SCALE_AUTO = -(2 ** 31)

STORAGE = {"f64": LBM_STORE_F64, "f32": LBM_STORE_F32, "f16": LBM_STORE_F16, "bf16": LBM_STORE_BF16}
COMPUTE = {"f64": LBM_COMPUTE_F64, "f32": LBM_COMPUTE_F32}
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


class LbmError(RuntimeError):
    def __init__(self, status, func, message):
        super().__init__(f"{func}: status {status}: {message}")
        self.status = status


class lbm_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("compute", ctypes.c_int32),
                ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double),
                ("s_q", ctypes.c_double), ("s_nu", ctypes.c_double),
                ("rho0", ctypes.c_double), ("u0x", ctypes.c_double), ("u0y", ctypes.c_double),
                ("scale_exp", ctypes.c_int32), ("flags", ctypes.c_int32)]


class lbm_launch(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("block_x", ctypes.c_int32),
                ("block_y", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("flags", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class lbm_pool_shape(ctypes.Structure):
    _fields_ = [("tile_cells", ctypes.c_int32), ("block", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32), ("seg_rows", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("flags", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_st = ctypes.c_int32

# name -> (restype, argtypes); the list mirrors include/lbm.h
SIGNATURES = {
    "lbm_status_string": (ctypes.c_char_p, [_st]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_s_from_nu": (ctypes.c_double, [ctypes.c_double]),
    "lbm_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(lbm_desc)]),
    "lbm_create": (_st, [ctypes.POINTER(lbm_desc), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "lbm_destroy": (_st, [_vp]),
    "lbm_set_stream": (_st, [_vp, _vp]),
    "lbm_get_desc": (_st, [_vp, ctypes.POINTER(lbm_desc)]),
    "lbm_init_equilibrium": (_st, [_vp, _vp, _vp, _vp]),
    "lbm_step": (_st, [_vp, ctypes.c_int64]),
    "lbm_read_moments": (_st, [_vp, _vp, _vp, _vp]),
    "lbm_diagnostics": (_st, [_vp, _dp]),
    "lbm_diagnostics_noalloc": (_st, [ctypes.POINTER(lbm_desc), _vp, _vp, _vp]),
    "lbm_project": (_st, [_vp, ctypes.c_int32, ctypes.c_int32, _vp]),
    "lbm_read_populations": (_st, [_vp, _vp]),
    "lbm_write_populations": (_st, [_vp, _vp]),
    "lbm_set_node_equilibrium": (_st, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double]),
    "lbm_state_bytes": (ctypes.c_size_t, [_vp]),
    "lbm_save_state": (_st, [_vp, _vp]),
    "lbm_load_state": (_st, [_vp, _vp, ctypes.c_int64]),
    "lbm_time": (ctypes.c_int64, [_vp]),
    "lbm_get_launch": (_st, [_vp, ctypes.POINTER(lbm_launch)]),
    "lbm_set_launch": (_st, [_vp, ctypes.POINTER(lbm_launch)]),
    "lbm_tune": (_st, [_vp, ctypes.c_int32, ctypes.POINTER(lbm_launch), _dp]),
    "lbm_time_launches": (_st, [_vp, ctypes.c_int32, _dp]),
    "lbm_steps_per_launch": (ctypes.c_int32, [ctypes.c_void_p]),
    "lbm_step_launches": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int64]),
    "lbm_pool_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "lbm_pool_create": (_st, [_vp, ctypes.c_size_t, _vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_vp)]),
    "lbm_pool_destroy": (_st, [_vp]),
    "lbm_pool_add": (_st, [_vp, _vp, ctypes.c_int64]),
    "lbm_pool_remove": (_st, [_vp, _vp]),
    "lbm_pool_step": (_st, [_vp, ctypes.c_int64]),
    "lbm_pool_poll": (_st, [_vp, ctypes.POINTER(_vp), ctypes.c_int32, ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_int32)]),
    "lbm_pool_members": (ctypes.c_int32, [_vp]),
    "lbm_pool_remaining": (ctypes.c_int64, [_vp, _vp]),
    "lbm_pool_get_shape": (_st, [_vp, ctypes.POINTER(lbm_pool_shape)]),
    "lbm_pool_set_shape": (_st, [_vp, ctypes.POINTER(lbm_pool_shape)]),
    "lbm_pool_time_launches": (_st, [_vp, ctypes.c_int32, _dp]),
    "lbm_pool_tune": (_st, [_vp, ctypes.c_int32, ctypes.POINTER(lbm_pool_shape), _dp]),
}


def load():
    """Loads liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                           f"g.build()'` (the GPU path has no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, func):
    if status != LBM_OK:
        lib = load()
        raise LbmError(status, func, lib.lbm_last_error().decode())
    return status


# ---- thin wrappers with the C names -------------------------------------------

def lbm_status_string(s):
    return load().lbm_status_string(s).decode()


def lbm_last_error():
    return load().lbm_last_error().decode()


def lbm_s_from_nu(nu):
    return load().lbm_s_from_nu(float(nu))


def lbm_workspace_bytes(desc):
    return int(load().lbm_workspace_bytes(ctypes.byref(desc)))


def lbm_create(desc, dev_ws, ws_bytes, stream):
    h = _vp()
    check(load().lbm_create(ctypes.byref(desc), _vp(dev_ws), ws_bytes, _vp(stream), ctypes.byref(h)), "lbm_create")
    return h


def lbm_destroy(h):
    check(load().lbm_destroy(h), "lbm_destroy")


def lbm_set_stream(h, stream):
    check(load().lbm_set_stream(h, _vp(stream)), "lbm_set_stream")


def lbm_get_desc(h):
    d = lbm_desc()
    check(load().lbm_get_desc(h, ctypes.byref(d)), "lbm_get_desc")
    return d


def lbm_init_equilibrium(h, rho, ux, uy):
    check(load().lbm_init_equilibrium(h, _vp(rho), _vp(ux), _vp(uy)), "lbm_init_equilibrium")


def lbm_step(h, n):
    check(load().lbm_step(h, int(n)), "lbm_step")


def lbm_read_moments(h, rho, ux, uy):
    check(load().lbm_read_moments(h, _vp(rho), _vp(ux), _vp(uy)), "lbm_read_moments")


def lbm_diagnostics(h):
    """Returns (status, [mass, momx, momy, nonfinite]); never raises for LBM_E_NONFINITE."""
    out = (ctypes.c_double * 4)()
    s = load().lbm_diagnostics(h, out)
    if s not in (LBM_OK, LBM_E_NONFINITE):
        check(s, "lbm_diagnostics")
    return s, [out[k] for k in range(4)]


def lbm_diagnostics_noalloc(desc, dev_state, dev_out, stream):
    """Enqueues the diagnostics of a raw state into dev_out (4 doubles on the
    device); allocates nothing."""
    check(load().lbm_diagnostics_noalloc(ctypes.byref(desc), _vp(dev_state), _vp(dev_out), _vp(stream)),
          "lbm_diagnostics_noalloc")


def lbm_project(h, mx, my, dev_out):
    check(load().lbm_project(h, int(mx), int(my), _vp(dev_out)), "lbm_project")


def lbm_read_populations(h, dev_f):
    check(load().lbm_read_populations(h, _vp(dev_f)), "lbm_read_populations")


def lbm_write_populations(h, dev_f):
    check(load().lbm_write_populations(h, _vp(dev_f)), "lbm_write_populations")


def lbm_set_node_equilibrium(h, x, y, rho, ux, uy):
    check(load().lbm_set_node_equilibrium(h, int(x), int(y), float(rho), float(ux), float(uy)),
          "lbm_set_node_equilibrium")


def lbm_state_bytes(h):
    return int(load().lbm_state_bytes(h))


def lbm_save_state(h, dev_dst):
    check(load().lbm_save_state(h, _vp(dev_dst)), "lbm_save_state")


def lbm_load_state(h, dev_src, t):
    check(load().lbm_load_state(h, _vp(dev_src), int(t)), "lbm_load_state")


def lbm_time(h):
    return int(load().lbm_time(h))


def lbm_get_launch(h):
    c = lbm_launch()
    check(load().lbm_get_launch(h, ctypes.byref(c)), "lbm_get_launch")
    return c


def lbm_set_launch(h, cfg):
    check(load().lbm_set_launch(h, ctypes.byref(cfg)), "lbm_set_launch")


def lbm_tune(h, reps):
    c = lbm_launch()
    us = ctypes.c_double()
    check(load().lbm_tune(h, int(reps), ctypes.byref(c), ctypes.byref(us)), "lbm_tune")
    return c, us.value


def lbm_time_launches(h, n):
    us = ctypes.c_double()
    check(load().lbm_time_launches(h, int(n), ctypes.byref(us)), "lbm_time_launches")
    return us.value


def lbm_steps_per_launch(cfg):
    return int(load().lbm_steps_per_launch(ctypes.byref(cfg)))


def lbm_step_launches(h, n):
    return int(load().lbm_step_launches(h, int(n)))


# ---- pools ----------------------------------------------------------------------

def lbm_pool_workspace_bytes(max_members, max_tiles):
    return int(load().lbm_pool_workspace_bytes(int(max_members), int(max_tiles)))


def lbm_pool_create(dev_ws, ws_bytes, stream, max_members, max_tiles):
    h = _vp()
    check(load().lbm_pool_create(_vp(dev_ws), ws_bytes, _vp(stream), int(max_members), int(max_tiles),
                                 ctypes.byref(h)), "lbm_pool_create")
    return h


def lbm_pool_destroy(p):
    check(load().lbm_pool_destroy(p), "lbm_pool_destroy")


def lbm_pool_add(p, lat, nsteps):
    check(load().lbm_pool_add(p, lat, int(nsteps)), "lbm_pool_add")


def lbm_pool_remove(p, lat):
    check(load().lbm_pool_remove(p, lat), "lbm_pool_remove")


def lbm_pool_step(p, nsteps):
    check(load().lbm_pool_step(p, int(nsteps)), "lbm_pool_step")


def lbm_pool_poll(p, cap, wait=False):
    """Returns the list of finished lattice handles (as integers)."""
    arr = (_vp * max(1, cap))()
    n = ctypes.c_int32()
    check(load().lbm_pool_poll(p, arr, int(cap), 1 if wait else 0, ctypes.byref(n)), "lbm_pool_poll")
    return [arr[i] for i in range(n.value)]


def lbm_pool_members(p):
    return int(load().lbm_pool_members(p))


def lbm_pool_remaining(p, lat):
    return int(load().lbm_pool_remaining(p, lat))


def lbm_pool_get_shape(p):
    s = lbm_pool_shape()
    check(load().lbm_pool_get_shape(p, ctypes.byref(s)), "lbm_pool_get_shape")
    return s


def lbm_pool_set_shape(p, shape):
    check(load().lbm_pool_set_shape(p, ctypes.byref(shape)), "lbm_pool_set_shape")


def lbm_pool_time_launches(p, reps):
    us = ctypes.c_double()
    check(load().lbm_pool_time_launches(p, int(reps), ctypes.byref(us)), "lbm_pool_time_launches")
    return us.value


def lbm_pool_tune(p, reps):
    s = lbm_pool_shape()
    us = ctypes.c_double()
    check(load().lbm_pool_tune(p, int(reps), ctypes.byref(s), ctypes.byref(us)), "lbm_pool_tune")
    return s, us.value
