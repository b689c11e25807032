"""Precision study on the full 8192 x 8192 multi-pulse workload (1000 steps,
Lallemand-Luo rates with nu = 1e-3, 16 seeded Gaussian pulses of amplitude
1e-5..1e-3 and half-width 3..12 cells).

* The FP64 run is checked against the oracle on sampled outputs: a cell's
  value after T steps depends only on cells within distance T, so the oracle
  run on a periodic window of side 2T + 1 + 2r around a block reproduces that
  (2r + 1)^2 block exactly (pinned on the CPU by
  test_window_run_reproduces_the_centre_of_a_larger_periodic_run).
* Every reduced-precision storage is compared with the FP64 run over the
  whole lattice and with the oracle on the same sampled block: FP64 storage
  with FP32 collide and FP32 storage within 1e-5 A; FP16 and BF16 within the
  rounding bound 3 u sqrt(T) A (u = 2^-11, 2^-8).
"""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from oracle import linear

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_pulses8192_precision_and_sampled_oracle_parity():
    from paper_1107_4543_amd import Lattice
    w = lbm_inputs.WORKLOADS["pulses8192"]
    nx, ny, T = w["nx"], w["ny"], w["steps"]
    ll = lbm_inputs.PRESETS["LL"]
    s = [ll["s_e"], ll["s_eps"], ll["s_q"], float(linear.s_from_nu(w["nu"]))]
    specs = lbm_inputs.random_pulse_specs(nx, ny, w["seed"], w["count"])
    dev = "cuda:0"
    fields = lbm_inputs.pulses_field_torch(nx, ny, specs, dev)
    A = float((fields[0] - 1.0).abs().max())

    ref = Lattice(nx, ny, *s, storage="f64", device=dev).init(*fields).step(T)
    rho_ref = ref.moments()[0]

    # sampled parity of the FP64 run: block of (2r+1)^2 cells around the
    # strongest pulse, oracle on a periodic window of side 2T + 1 + 2r
    r = 6
    p = max(specs, key=lambda q: q.amplitude)
    gx, gy = int(p.cx) % nx, int(p.cy) % ny
    side = 2 * T + 1 + 2 * r
    x0, y0 = gx - T - r, gy - T - r
    win = oracle.run(oracle.init(*lbm_inputs.pulses_window(nx, ny, specs, x0, y0, side)), s, T)
    blk = win[:, T:T + 2 * r + 1, T:T + 2 * r + 1]
    ys = torch.tensor((y0 + np.arange(T, T + 2 * r + 1)) % ny, device=dev)
    xs = torch.tensor((x0 + np.arange(T, T + 2 * r + 1)) % nx, device=dev)
    f = ref.populations()
    got = f[:, ys][:, :, xs].cpu().numpy()
    del f
    assert np.max(np.abs(got - blk)) <= 1e-12 * np.max(np.abs(blk))
    rho_blk, ux_blk, uy_blk = oracle.moments(np.ascontiguousarray(blk))
    # velocity amplitude: an acoustic fluctuation of density amplitude A moves
    # the fluid at c_s A (the input itself is at rest)
    Au = max(float(np.max(np.abs(ux_blk))), float(np.max(np.abs(uy_blk))), lbm_inputs.CS * A)

    errs = {}
    for storage, compute, unit in [("f64", "f32", None), ("f32", "f32", None),
                                   ("f16", "f32", 2.0 ** -11), ("bf16", "f32", 2.0 ** -8)]:
        lat = Lattice(nx, ny, *s, storage=storage, compute=compute, device=dev).init(*fields).step(T)
        rho, ux, uy = lat.moments()
        # the sampled block against the oracle
        bound = 1e-5 if unit is None else 3.0 * unit * np.sqrt(T)
        b_rho = rho[ys][:, xs].cpu().numpy()
        e_blk = float(np.max(np.abs(b_rho - rho_blk))) / A
        print(f"{storage}/{compute}: block vs oracle Linf/A = {e_blk:.3e}")
        assert e_blk <= bound, (storage, compute, e_blk)
        if unit is None:
            e_u = max(float(np.max(np.abs(ux[ys][:, xs].cpu().numpy() - ux_blk))),
                      float(np.max(np.abs(uy[ys][:, xs].cpu().numpy() - uy_blk))))
            assert e_u <= 1e-5 * Au, (storage, compute, e_u / Au)
        del ux, uy
        d = rho - rho_ref
        e_inf = float(d.abs().max()) / A
        e_l2 = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(rho_ref - 1.0))
        errs[(storage, compute)] = (e_inf, e_l2)
        print(f"{storage}/{compute}: Linf/A = {e_inf:.3e}  L2 = {e_l2:.3e}")
        assert e_inf <= bound, (storage, compute, e_inf)
        del lat, rho, d
