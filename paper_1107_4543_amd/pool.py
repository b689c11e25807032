"""``Pool``: many lattices advanced together by the library's batched kernels
(one persistent launch per storage class and step, the step loop replayed as
a HIP graph).  Marshalling only; see include/lbm.h for the semantics."""
import torch

from . import _lib


class Pool:
    def __init__(self, max_members=256, max_tiles=1 << 16, device="cuda", stream=None):
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = _lib.lbm_pool_workspace_bytes(max_members, max_tiles)
        if nbytes == 0:
            raise _lib.LbmError(_lib.LBM_E_INVAL, "lbm_pool_workspace_bytes", "size out of range")
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._h = _lib.lbm_pool_create(self._ws.data_ptr(), nbytes, self.stream.cuda_stream,
                                       max_members, max_tiles)
        self.max_members = max_members
        self._members = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.lbm_pool_destroy(self._h)
            self._h = None
            self._members.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, lat, nsteps):
        _lib.lbm_pool_add(self._h, lat.handle, nsteps)
        self._members[lat.handle.value] = lat
        return self

    def remove(self, lat):
        _lib.lbm_pool_remove(self._h, lat.handle)
        self._members.pop(lat.handle.value, None)
        return self

    def step(self, nsteps):
        _lib.lbm_pool_step(self._h, nsteps)
        return self

    def poll(self, wait=False, cap=None):
        """Finished lattices (they leave the pool)."""
        hs = _lib.lbm_pool_poll(self._h, cap or self.max_members, wait)
        return [self._members.pop(h) for h in hs]

    @property
    def members(self):
        return _lib.lbm_pool_members(self._h)

    def remaining(self, lat):
        return _lib.lbm_pool_remaining(self._h, lat.handle)

    @property
    def shape(self):
        return _lib.lbm_pool_get_shape(self._h).as_dict()

    def set_shape(self, tile_cells=256, block=512, grid=4096, graph_steps=256, steps_per_launch=7, seg_rows=96,
                  waves=4, flags=32):
        """steps_per_launch 1 advances every member one step per launch over
        tiles of about tile_cells cells; 2, 4, 5, 6 or 7 uses strip tasks of the
        several-steps-per-pass kernel (seg_rows rows, `waves` waves per
        workgroup, kernel flags 0, 2, 4 or 12 as for Lattice.set_launch, or
        32 / 34 with four waves: one workgroup per strip task, halo columns
        shared through LDS; 96 / 98: the same with two-wave workgroups for
        left-over columns that fit them)."""
        _lib.lbm_pool_set_shape(self._h, _lib.lbm_pool_shape(tile_cells, block, grid, graph_steps, steps_per_launch,
                                                             seg_rows, waves, flags))
        return self

    def time_launches(self, reps=5):
        """Microseconds per launch (steps_per_launch steps of every member)."""
        return _lib.lbm_pool_time_launches(self._h, reps)

    def tune(self, reps=5):
        """Selects the shape with the least time per step; returns (shape, us per step)."""
        s, us = _lib.lbm_pool_tune(self._h, reps)
        return s.as_dict(), us
