"""The allocation-free diagnostics entry point (lbm_diagnostics_noalloc)
against lbm_diagnostics through the C ABI: the same sums, bit for bit, on
two calls in a row (the second on a smaller lattice, so stale partial sums
of the first call would show), for every storage type."""
import numpy as np
import pytest
import torch

import lbm_inputs

pytestmark = pytest.mark.gpu


def _lattice(nx, ny, storage, seed):
    from paper_1107_4543_amd import Lattice
    rng = np.random.default_rng(seed)
    rho = 1.0 + 1e-3 * rng.standard_normal((ny, nx))
    ux = 0.02 + 1e-3 * rng.standard_normal((ny, nx))
    uy = 1e-3 * rng.standard_normal((ny, nx))
    lat = Lattice(nx, ny, 1.3, 1.2, 1.7, 1.85, storage=storage, u0=(0.02, 0.0), device="cuda:0")
    return lat.init(rho, ux, uy).step(23)


def _noalloc(lat):
    from paper_1107_4543_amd import _lib
    d = _lib.lbm_get_desc(lat.handle)              # explicit scale_exp once initialised
    buf, t = lat.save_state()
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda:0")
    with torch.cuda.stream(lat.stream):
        _lib.lbm_diagnostics_noalloc(d, buf.data_ptr(), out.data_ptr(), lat.stream.cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().tolist()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_noalloc_diagnostics_equal_the_workspace_ones_on_two_calls(storage):
    big = _lattice(300, 257, storage, 1)            # 77,100 cells: every partial row in use
    small = _lattice(37, 5, storage, 2)             # 185 cells: one partial row
    for lat in (big, small):
        st, ref = lat.diagnostics()
        assert st == 0
        got = _noalloc(lat)
        assert got == ref, (storage, lat.nx, lat.ny, got, ref)
        assert any(v != 0.0 for v in got[:3])


def test_noalloc_rejects_bad_arguments():
    from paper_1107_4543_amd import _lib
    lat = _lattice(40, 30, "f16", 3)
    d = _lib.lbm_get_desc(lat.handle)
    buf, _ = lat.save_state()
    out = torch.empty(4, dtype=torch.float64, device="cuda:0")
    d.scale_exp = _lib.LBM_SCALE_AUTO               # the state's scale is required for 16-bit storage
    with pytest.raises(_lib.LbmError) as e:
        _lib.lbm_diagnostics_noalloc(d, buf.data_ptr(), out.data_ptr(), lat.stream.cuda_stream)
    assert e.value.status == _lib.LBM_E_INVAL
    d = _lib.lbm_get_desc(lat.handle)
    d.nx = 1 << 30                                   # beyond the library's lattice size limit
    with pytest.raises(_lib.LbmError) as e:
        _lib.lbm_diagnostics_noalloc(d, buf.data_ptr(), out.data_ptr(), lat.stream.cuda_stream)
    assert e.value.status == _lib.LBM_E_INVAL
    with pytest.raises(_lib.LbmError):
        _lib.lbm_diagnostics_noalloc(_lib.lbm_get_desc(lat.handle), buf.data_ptr(), 0, lat.stream.cuda_stream)
