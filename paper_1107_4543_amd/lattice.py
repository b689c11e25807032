"""``Lattice``: one periodic D2Q9 MRT lattice on the GPU.

PyTorch supplies the device workspace and the stream; every operation is a
call into the C ABI (``_lib``), which enqueues the library's own HIP kernels.
"""
import numpy as np
import torch

from . import _lib


def _dev_f64(a, device):
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=torch.float64)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)
    return t.contiguous()


class Lattice:
    """A lattice of nx x ny cells with relaxation rates (s_e, s_eps, s_q, s_nu)
    (Sec. 2.3 of the paper), stored as deviations about f^eq(rho0, u0).

    storage: "f64" | "f32" | "f16" | "bf16"; compute: "f64" | "f32" (default:
    f64 for f64 storage, else f32).  ``stream``: a torch.cuda.Stream (default:
    the current stream of ``device``)."""

    def __init__(self, nx, ny, s_e, s_eps, s_q, s_nu, storage="f32", compute=None,
                 rho0=1.0, u0=(0.0, 0.0), scale_exp=None, device="cuda", stream=None):
        if compute is None:
            compute = "f64" if storage == "f64" else "f32"
        self.device = torch.device(device)
        self.nx, self.ny = int(nx), int(ny)
        self.storage, self.compute = storage, compute
        d = _lib.lbm_desc()
        d.nx, d.ny = self.nx, self.ny
        d.storage = _lib.STORAGE[storage]
        d.compute = _lib.COMPUTE[compute]
        d.s_e, d.s_eps, d.s_q, d.s_nu = float(s_e), float(s_eps), float(s_q), float(s_nu)
        d.rho0, d.u0x, d.u0y = float(rho0), float(u0[0]), float(u0[1])
        d.scale_exp = _lib.LBM_SCALE_AUTO if scale_exp is None else int(scale_exp)
        d.flags = 0
        self.desc = d
        nbytes = _lib.lbm_workspace_bytes(d)
        if nbytes == 0:
            raise _lib.LbmError(_lib.LBM_E_INVAL, "lbm_workspace_bytes", _lib.lbm_last_error())
        self.workspace_bytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._h = _lib.lbm_create(d, self._ws.data_ptr(), nbytes, self.stream.cuda_stream)

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- state ----------------------------------------------------------------
    def init(self, rho, ux, uy):
        """Equilibrium initialisation from [ny, nx] fields (numpy or torch)."""
        self._fields = [_dev_f64(a, self.device) for a in (rho, ux, uy)]
        for a in self._fields:
            if tuple(a.shape) != (self.ny, self.nx):
                raise ValueError(f"field shape {tuple(a.shape)} != {(self.ny, self.nx)}")
            if self.stream != torch.cuda.current_stream(self.device):
                self.stream.wait_stream(torch.cuda.current_stream(self.device))
                a.record_stream(self.stream)
        with torch.cuda.stream(self.stream):
            _lib.lbm_init_equilibrium(self._h, *(a.data_ptr() for a in self._fields))
        return self

    def step(self, n=1):
        _lib.lbm_step(self._h, n)
        return self

    @property
    def t(self):
        return _lib.lbm_time(self._h)

    @property
    def scale_exp(self):
        return _lib.lbm_get_desc(self._h).scale_exp

    def moments(self):
        """(rho, ux, uy) as [ny, nx] float64 device tensors (stream-ordered)."""
        with torch.cuda.stream(self.stream):
            out = [torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) for _ in range(3)]
            _lib.lbm_read_moments(self._h, *(a.data_ptr() for a in out))
        return tuple(out)

    def diagnostics(self):
        """(status, [sum rho', sum jx', sum jy', nonfinite])."""
        return _lib.lbm_diagnostics(self._h)

    def project(self, mx, my, out=None):
        """Complex FP64 projection of the population deviations on mode (mx, my);
        returns (or fills) a float64 device tensor of 18 values."""
        with torch.cuda.stream(self.stream):
            if out is None:
                out = torch.empty(18, dtype=torch.float64, device=self.device)
            _lib.lbm_project(self._h, mx, my, out.data_ptr())
        return out

    def populations(self):
        with torch.cuda.stream(self.stream):
            f = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.device)
            _lib.lbm_read_populations(self._h, f.data_ptr())
        return f

    def set_populations(self, f):
        f = _dev_f64(f, self.device)
        self._fpop = f
        with torch.cuda.stream(self.stream):
            _lib.lbm_write_populations(self._h, f.data_ptr())
        return self

    def set_node_equilibrium(self, x, y, rho, ux=0.0, uy=0.0):
        """Imposes f(x, y) = f^eq(rho, rho u) on one node (point source)."""
        _lib.lbm_set_node_equilibrium(self._h, x, y, rho, ux, uy)
        return self

    def save_state(self):
        with torch.cuda.stream(self.stream):
            buf = torch.empty(_lib.lbm_state_bytes(self._h), dtype=torch.uint8, device=self.device)
            _lib.lbm_save_state(self._h, buf.data_ptr())
        return buf, self.t

    def load_state(self, buf, t):
        self._loaded = buf
        with torch.cuda.stream(self.stream):
            _lib.lbm_load_state(self._h, buf.data_ptr(), t)
        return self

    # -- launch shape -----------------------------------------------------------
    @property
    def launch(self):
        return _lib.lbm_get_launch(self._h).as_dict()

    def set_launch(self, variant=0, block_x=64, block_y=4, rows=1, xcd_remap=1, flags=0):
        c = _lib.lbm_launch(variant, block_x, block_y, rows, xcd_remap, flags)
        _lib.lbm_set_launch(self._h, c)
        return self

    @property
    def steps_per_launch(self):
        """Steps one launch of the current shape advances."""
        return _lib.lbm_steps_per_launch(_lib.lbm_get_launch(self._h))

    def launches_for(self, n):
        """Kernel launches step(n) makes with the current shapes."""
        return _lib.lbm_step_launches(self._h, n)

    def tune(self, reps=10):
        """Selects the launch shape with the least time per step; returns
        (shape, microseconds per step)."""
        c, us = _lib.lbm_tune(self._h, reps)
        return c.as_dict(), us

    def time_launches(self, n):
        """Microseconds per launch of the current shape (steps_per_launch steps)."""
        return _lib.lbm_time_launches(self._h, n)
