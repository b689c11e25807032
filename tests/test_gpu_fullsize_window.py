"""Full-size oracle parity of the benched several-steps kernels in both
directions: a 4096 x 4096 lattice with 16 seeded Gaussian pulses (fields
that vary along x and y) on the mean flow u_x = 0.1 c_s with the Table 5
group A rates, run with each storage type's recorded default launch shape
(the one bench.py times: for FP32 seven steps per pass, workgroups of four
waves sharing their halo columns, strips of 244 columns and 92-row segments),
compared with the FP64 oracle on sampled blocks.

A cell's value after T steps depends only on cells within distance T, so the
oracle run on a periodic window of side 2T + 1 + 2r reproduces a (2r + 1)^2
block of the full run exactly (pinned on the CPU by
test_window_run_reproduces_the_centre_of_a_larger_periodic_run).  The blocks
straddle the places where the kernel's work is cut: strip edges, segment
edges and the lattice's periodic wrap.
Tolerances: FP64 to 1e-12 of the density (and the velocity, momentum-relative);
FP32 within 1e-5 A on the density and 1e-5 A_u on the velocity; FP16 and BF16
storage within the rounding bound 3 u sqrt(T) A.
"""
import numpy as np
import pytest
import torch

import bench
import lbm_inputs
import oracle

pytestmark = pytest.mark.gpu

N = 4096
T = 147                       # 21 seven-step launches
R = 5                         # blocks of 11 x 11 cells
# block centres: strip edges (x = 244 k for the FP32 shape; 52 k of the
# one-wave strips), segment edges (y = 92 k; 69 k for FP16/BF16), the corner
# (periodic wrap in x and y), interior cells
CENTRES = [(244 * 3, 92 * 5), (244 * 9 + 1, 69 * 12 - 1), (0, 0), (N - 1, 2000), (52 * 40, 168 * 12),
           (1234, 3210)]
# the launch shapes bench.py times (the recorded defaults for each storage type)
LAUNCH = {k: tuple(int(x) for x in v.split(",")) for k, v in bench.DEFAULT_LAUNCH.items()}


def _rates():
    t = lbm_inputs.PRESETS["T5A"]
    return [t["s_e"], t["s_eps"], t["s_q"], t["s_nu"]]


@pytest.fixture(scope="module")
def workload():
    u0x = 0.1 * lbm_inputs.CS
    specs = lbm_inputs.random_pulse_specs(N, N, seed=77, count=16, amp_range=(1e-5, 1e-3))
    # put pulses on the sampled blocks so that every block sees a signal
    assert len(specs) >= len(CENTRES)
    for k, (cx, cy) in enumerate(CENTRES):
        specs[k].cx, specs[k].cy = cx + 0.3, cy - 0.4
    s = _rates()
    side = 2 * T + 1 + 2 * R
    blocks = []
    for cx, cy in CENTRES:
        x0, y0 = cx - T - R, cy - T - R
        rho, ux, uy = lbm_inputs.pulses_window(N, N, specs, x0, y0, side)
        win = oracle.run(oracle.init(rho, ux + u0x, uy), s, T)
        blk = np.ascontiguousarray(win[:, T:T + 2 * R + 1, T:T + 2 * R + 1])
        ys = (y0 + np.arange(T, T + 2 * R + 1)) % N
        xs = (x0 + np.arange(T, T + 2 * R + 1)) % N
        blocks.append((ys, xs, oracle.moments(blk)))
    return specs, u0x, s, blocks


@pytest.mark.timeout(600)
@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_benched_shape_matches_window_oracle(workload, storage):
    from paper_1107_4543_amd import Lattice
    specs, u0x, s, blocks = workload
    dev = "cuda:0"
    rho, ux, uy = lbm_inputs.pulses_field_torch(N, N, specs, dev)
    ux += u0x
    A = float((rho - 1.0).abs().max())
    lat = Lattice(N, N, *s, storage=storage, u0=(u0x, 0.0), device=dev)
    v, bx, by, rows, remap, flags = LAUNCH[storage]
    lat.set_launch(variant=v, block_x=bx, block_y=by, rows=rows, xcd_remap=remap, flags=flags)
    assert lat.steps_per_launch == v - 6
    lat.init(rho, ux, uy)
    del rho, ux, uy
    lat.step(T)
    assert lat.t == T
    r, u, w = lat.moments()
    unit = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}.get(storage)
    worst = 0.0
    for ys, xs, (rb, ub, wb) in blocks:
        yi, xi = torch.tensor(ys, device=dev), torch.tensor(xs, device=dev)
        gr = r[yi][:, xi].cpu().numpy()
        e = float(np.max(np.abs(gr - rb))) / A
        worst = max(worst, e)
        if storage == "f64":
            eu = max(float(np.max(np.abs(u[yi][:, xi].cpu().numpy() - ub))),
                     float(np.max(np.abs(w[yi][:, xi].cpu().numpy() - wb))))
            assert float(np.max(np.abs(gr - rb))) <= 1e-12 * float(np.max(np.abs(rb))), (storage, ys[0], xs[0])
            assert eu <= 1e-12 * float(np.max(np.abs(rb))), (storage, ys[0], xs[0])
        elif unit is None:
            Au = lbm_inputs.CS * A
            eu = max(float(np.max(np.abs(u[yi][:, xi].cpu().numpy() - ub))),
                     float(np.max(np.abs(w[yi][:, xi].cpu().numpy() - wb))))
            assert e <= 1e-5, (storage, ys[0], xs[0], e)
            assert eu <= 1e-5 * Au, (storage, ys[0], xs[0], eu / Au)
        else:
            assert e <= 3.0 * unit * np.sqrt(T), (storage, ys[0], xs[0], e)
    print(f"{storage}: worst block error / A = {worst:.3e}")
