"""Batched stepping (pools) on the GPU: every member advances exactly its own
number of steps and ends bit-identical to the same lattice stepped alone;
membership changes between steps; parity with the oracle; error paths."""
import numpy as np
import pytest
import torch

import lbm_inputs
import oracle
from oracle import linear

pytestmark = pytest.mark.gpu


def make(nx, ny, s, storage="f32", seed=0, u0=(0.0, 0.0), amp=1e-3):
    from paper_1107_4543_amd import Lattice
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.standard_normal((ny, nx))
    ux = u0[0] + amp * rng.standard_normal((ny, nx))
    uy = u0[1] + amp * rng.standard_normal((ny, nx))
    lat = Lattice(nx, ny, *s, storage=storage, u0=u0, device="cuda:0")
    lat.init(rho, ux, uy)
    return lat, (rho, ux, uy)


def twin(lat, fields, s):
    from paper_1107_4543_amd import Lattice
    t = Lattice(lat.nx, lat.ny, *s, storage=lat.storage, u0=(lat.desc.u0x, lat.desc.u0y), device="cuda:0",
                scale_exp=lat.scale_exp)
    return t.init(*fields)


SETS = [[1.64, 1.54, 1.9, 1.98], [1.3, 1.1, 1.7, 1.85], [1.99, 1.962820428, 1.992761413, 1.999960001],
        [1.2, 1.5, 1.4, 1.6], [1.5, 1.5, 1.5, 1.5], [1.8, 1.2, 1.95, 1.7]]
SIZES = [(64, 64), (100, 37), (257, 64), (33, 190), (1, 9), (128, 128)]
STORES = ["f32", "f16", "f64", "bf16", "f32", "f32"]
STEPS = [37, 100, 0, 64, 5, 91]
# one step per launch, and T-step strip tasks (T = 2, 4, 5, 6, 7) with their
# one-step launches for left-over steps; with graph_steps 16 the recorded
# loops are T 2^m steps (16, 10, 12 or 14) and powers of two below T, recorded
# with and without one-step launches as the members' counts require
SCHEDULES = [dict(steps_per_launch=1), dict(steps_per_launch=2, seg_rows=16, waves=2, flags=0),
             dict(steps_per_launch=4, seg_rows=32, waves=4, flags=2),
             dict(steps_per_launch=4, seg_rows=7, waves=1, flags=12),
             dict(steps_per_launch=5, seg_rows=16, waves=4, flags=2),
             dict(steps_per_launch=6, seg_rows=9, waves=2, flags=0),
             dict(steps_per_launch=7, seg_rows=13, waves=4, flags=2)]


@pytest.mark.parametrize("sched", SCHEDULES)
def test_members_match_alone_bitwise_with_own_step_counts(sched):
    from paper_1107_4543_amd.pool import Pool
    pool = Pool(max_members=16, max_tiles=4096)
    pool.set_shape(tile_cells=512, block=256, grid=64, graph_steps=16, **sched)
    lats, twins = [], []
    for i, ((nx, ny), s, st, n) in enumerate(zip(SIZES, SETS, STORES, STEPS)):
        lat, f = make(nx, ny, s, st, seed=i, u0=(0.02 * (i % 2), 0.0))
        lat.step(3)                                  # members need not start at t = 0
        pool.add(lat, n)
        lats.append(lat)
        twins.append(twin(lat, f, s).step(3 + n))
    pool.step(60)
    torch.cuda.synchronize()
    done = {id(l) for l in pool.poll()}
    for lat, n in zip(lats, STEPS):
        assert (id(lat) in done) == (n <= 60)
    pool.step(1000)
    torch.cuda.synchronize()
    rest = pool.poll(wait=True)
    while pool.members:
        rest += pool.poll(wait=True)
    for lat, tw, n in zip(lats, twins, STEPS):
        assert lat.t == 3 + n
        assert torch.equal(lat.populations(), tw.populations()), (lat.nx, lat.ny, lat.storage)
    pool.close()


@pytest.mark.parametrize("sched", SCHEDULES)
def test_continuous_membership_and_remove(sched):
    from paper_1107_4543_amd import _lib
    from paper_1107_4543_amd.pool import Pool
    pool = Pool(max_members=4, max_tiles=1024)
    pool.set_shape(tile_cells=1024, block=128, grid=32, graph_steps=8, **sched)
    s = SETS[0]
    a, fa = make(96, 40, s, "f32", seed=1)
    b, fb = make(50, 70, s, "f32", seed=2)
    c, fc = make(70, 20, s, "f64", seed=3)
    pool.add(a, 50)
    pool.step(20)                                     # several recorded loops
    pool.add(b, 30)                                   # joins while a is in flight
    with pytest.raises(_lib.LbmError) as e:
        a.step(1)
    assert e.value.status == _lib.LBM_E_STATE
    with pytest.raises(_lib.LbmError):
        pool.add(a, 1)
    pool.step(13)
    pool.add(c, 40)
    pool.step(11)
    pool.remove(c)                                    # leaves after 11 of 40 steps
    assert c.t == 11
    assert pool.remaining(a) == 50 - 44 and pool.remaining(b) == 30 - 24
    pool.step(100)
    out = []
    while pool.members:
        out += pool.poll(wait=True)
    assert {id(x) for x in out} == {id(a), id(b)}
    assert a.t == 50 and b.t == 30
    for lat, f, n in [(a, fa, 50), (b, fb, 30), (c, fc, 11)]:
        assert torch.equal(lat.populations(), twin(lat, f, s).step(n).populations())
    c.step(2)                                         # usable again after leaving
    assert c.t == 13
    pool.close()


@pytest.mark.parametrize("sched", SCHEDULES)
def test_pool_member_parity_with_oracle_fp64(sched):
    from paper_1107_4543_amd.pool import Pool
    pool = Pool(max_members=4, max_tiles=512)
    pool.set_shape(tile_cells=256, block=64, grid=16, graph_steps=10, **sched)
    s = [1.64, 1.54, 1.9, float(linear.s_from_nu(1e-3))]
    lat, (rho, ux, uy) = make(48, 30, s, "f64", seed=7, u0=(0.03, 0.0))
    pool.add(lat, 77)
    pool.step(77)
    assert pool.poll(wait=True) == [lat]
    ref = oracle.run(oracle.init(rho, ux, uy), s, 77)
    f = lat.populations().cpu().numpy()
    assert np.max(np.abs(f - ref)) <= 1e-12 * np.max(np.abs(ref))
    pool.close()


def test_pool_tune_and_timing_leave_states_unchanged():
    from paper_1107_4543_amd.pool import Pool
    pool = Pool(max_members=8, max_tiles=8192)
    lats = []
    for i in range(3):
        lat, _ = make(128 + 32 * i, 96, SETS[i], "f32", seed=10 + i)
        pool.add(lat, 10)
        lats.append(lat)
    shape, us = pool.tune(reps=2)
    assert us > 0 and shape["tile_cells"] >= 256
    pool.time_launches(2)
    for lat in lats:
        pool.remove(lat)
        assert lat.t == 0
    # states untouched: stepping now equals stepping fresh twins
    for i, lat in enumerate(lats):
        _, f = make(128 + 32 * i, 96, SETS[i], "f32", seed=10 + i)
        assert torch.equal(lat.step(4).populations(), twin(lat, f, SETS[i]).step(4).populations())
    pool.close()


def test_full_batch_of_256_lattices_matches_alone_on_a_sample():
    # The batched workload: 256 lattices of log-uniform sides in [64, 1024],
    # sampled rates (kept only if linearly stable), one pulse each, 500 steps.
    from paper_1107_4543_amd import Lattice
    from paper_1107_4543_amd import stability
    from paper_1107_4543_amd.pool import Pool
    w = lbm_inputs.WORKLOADS["batch256"]
    specs = lbm_inputs.batch_specs(w["seed"], w["count"], steps=w["steps"], accept=stability.stable)
    pool = Pool(max_members=256, max_tiles=1 << 18)
    lats = []
    for sp in specs:
        lat = Lattice(sp.nx, sp.ny, *stability.rates(sp.relax), storage="f32", device="cuda:0")
        lat.init(*sp.fields())
        pool.add(lat, sp.steps)
        lats.append(lat)
    pool.step(w["steps"])
    got = []
    while pool.members:
        got += pool.poll(wait=True)
    assert len(got) == 256
    for j in range(0, 256, 37):
        sp = specs[j]
        alone = Lattice(sp.nx, sp.ny, *stability.rates(sp.relax), storage="f32", device="cuda:0")
        alone.init(*sp.fields()).step(sp.steps)
        assert torch.equal(lats[j].populations(), alone.populations()), j
        st, d = lats[j].diagnostics()
        assert st == 0
    pool.close()


# Shared-halo tables (flags bit 5): every strip task is one workgroup of four
# waves that pass their halo values through LDS.  Widths around the
# workgroup strip (244 columns at T = 7 for 32-bit storage): an exact strip,
# strips plus a narrow remainder, members narrower than a strip (whose lanes
# wrap around the lattice) and a one-column member.  Flags 32 / 34 put
# left-over columns in a narrower four-wave strip, 96 / 98 in a two-wave one
# when they fit it.
WG_SIZES = [(600, 70), (200, 45), (257, 64), (64, 64), (1, 9), (490, 33), (244, 20), (31, 150), (1100, 12)]
WG_STORES = ["f32", "f16", "f32", "bf16", "f32", "f64", "f32", "f16", "f32"]
WG_STEPS = [37, 50, 23, 64, 5, 44, 71, 30, 19]
WG_SCHEDULES = [dict(steps_per_launch=7, seg_rows=13, waves=4, flags=32),
                   dict(steps_per_launch=7, seg_rows=40, waves=4, flags=34),
                   dict(steps_per_launch=6, seg_rows=9, waves=4, flags=32),
                   dict(steps_per_launch=4, seg_rows=16, waves=4, flags=34),
                   dict(steps_per_launch=2, seg_rows=5, waves=4, flags=32),
                   dict(steps_per_launch=7, seg_rows=13, waves=4, flags=96),
                   dict(steps_per_launch=7, seg_rows=40, waves=4, flags=98),
                   dict(steps_per_launch=6, seg_rows=9, waves=4, flags=96),
                   dict(steps_per_launch=4, seg_rows=16, waves=4, flags=98),
                   dict(steps_per_launch=2, seg_rows=5, waves=4, flags=96)]


@pytest.mark.parametrize("sched", WG_SCHEDULES)
def test_shared_halo_tables_match_alone_bitwise(sched):
    from paper_1107_4543_amd.pool import Pool
    pool = Pool(max_members=16, max_tiles=1 << 14)
    # grid 32: a workgroup walks several tasks in turn
    pool.set_shape(tile_cells=512, block=256, grid=32, graph_steps=16, **sched)
    lats, twins = [], []
    for i, ((nx, ny), st, n) in enumerate(zip(WG_SIZES, WG_STORES, WG_STEPS)):
        s = SETS[i % len(SETS)]
        lat, f = make(nx, ny, s, st, seed=40 + i, u0=(0.02 * (i % 2), 0.0))
        lat.step(2)
        pool.add(lat, n)
        lats.append(lat)
        twins.append(twin(lat, f, s).step(2 + n))
    pool.step(30)
    pool.step(100)
    torch.cuda.synchronize()
    out = []
    while pool.members:
        out += pool.poll(wait=True)
    assert len(out) == len(lats)
    for lat, tw, n in zip(lats, twins, WG_STEPS):
        assert lat.t == 2 + n
        assert torch.equal(lat.populations(), tw.populations()), (lat.nx, lat.ny, lat.storage, sched)
    pool.close()


@pytest.mark.parametrize("flags", [32, 96])
def test_shared_halo_table_member_parity_with_oracle_fp64(flags):
    # 263 columns: one 244-column strip and 19 left over (a narrower
    # four-wave strip with flags 32, a two-wave one with 96)
    from paper_1107_4543_amd.pool import Pool
    pool = Pool(max_members=4, max_tiles=1024)
    pool.set_shape(tile_cells=256, block=64, grid=16, graph_steps=14, steps_per_launch=7, seg_rows=11, waves=4,
                   flags=flags)
    s = [1.64, 1.54, 1.9, float(linear.s_from_nu(1e-3))]
    lat, (rho, ux, uy) = make(263, 30, s, "f64", seed=8, u0=(0.03, 0.0))
    pool.add(lat, 33)
    pool.step(33)
    assert pool.poll(wait=True) == [lat]
    ref = oracle.run(oracle.init(rho, ux, uy), s, 33)
    f = lat.populations().cpu().numpy()
    assert np.max(np.abs(f - ref)) <= 1e-12 * np.max(np.abs(ref))
    pool.close()


def test_shared_halo_shapes_need_four_waves_and_the_halo_bit():
    # flag 32 tables run four-wave workgroups; bit 6 (two-wave workgroups for
    # left-over columns) only goes with them (96, 98)
    from paper_1107_4543_amd import _lib
    from paper_1107_4543_amd.pool import Pool
    pool = Pool(max_members=2, max_tiles=256)
    for waves in (1, 2, 3):
        for flags in (32, 96):
            with pytest.raises(_lib.LbmError) as e:
                pool.set_shape(steps_per_launch=7, seg_rows=64, waves=waves, flags=flags)
            assert e.value.status == _lib.LBM_E_INVAL
    for flags in (64, 66, 76):
        with pytest.raises(_lib.LbmError) as e:
            pool.set_shape(steps_per_launch=7, seg_rows=64, waves=4, flags=flags)
        assert e.value.status == _lib.LBM_E_INVAL
    for flags in (34, 96, 98):
        pool.set_shape(steps_per_launch=7, seg_rows=64, waves=4, flags=flags)
        assert pool.shape["flags"] == flags
    pool.close()


def test_shorter_segments_never_outgrow_the_tile_table():
    # A pool of 16-bit members that fills four workgroups per compute unit
    # cuts its strips at 0.75 x seg_rows, which makes more tasks than
    # lbm_pool_add counts (at seg_rows).  With the smallest tile table that
    # accepts two FP16 4096^2 members, the pool keeps seg_rows and steps;
    # the results equal the members' own runs.
    import torch
    from paper_1107_4543_amd import Lattice, _lib
    from paper_1107_4543_amd.pool import Pool
    s = SETS[0]
    nx = ny = 4096

    def fields(seed):
        rng = np.random.default_rng(seed)
        return [torch.as_tensor(a, device="cuda:0") for a in
                (1.0 + 1e-3 * rng.standard_normal((ny, nx)), 1e-3 * rng.standard_normal((ny, nx)),
                 1e-3 * rng.standard_normal((ny, nx)))]

    f = [fields(70), fields(71)]
    lats = [Lattice(nx, ny, *s, storage="f16", device="cuda:0", scale_exp=22).init(*f[i]) for i in range(2)]
    shape = dict(tile_cells=512, block=512, grid=4096, graph_steps=16, steps_per_launch=6, seg_rows=96, waves=4,
                 flags=34)

    def accepts(max_tiles):
        # members with steps to go count their tiles; nothing is stepped
        pool = Pool(max_members=4, max_tiles=max_tiles)
        pool.set_shape(**shape)
        added = []
        try:
            for lat in lats:
                pool.add(lat, 8)
                added.append(lat)
            return True
        except _lib.LbmError as e:
            assert e.status == _lib.LBM_E_NOMEM
            return False
        finally:
            for lat in added:
                pool.remove(lat)
            pool.close()

    lo, hi = 1, 1 << 18                       # accepts(hi), not accepts(lo)
    assert accepts(hi) and not accepts(lo)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if accepts(mid):
            hi = mid
        else:
            lo = mid
    pool = Pool(max_members=4, max_tiles=hi)
    pool.set_shape(**shape)
    for lat in lats:
        pool.add(lat, 8)
    pool.step(8)
    done = []
    while pool.members:
        done += pool.poll(wait=True)
    pool.close()
    assert len(done) == 2
    for i, lat in enumerate(lats):
        tw = Lattice(nx, ny, *s, storage="f16", device="cuda:0", scale_exp=22).init(*f[i]).step(8)
        assert lat.t == 8 and torch.equal(lat.populations(), tw.populations()), i
        tw.close()
        lat.close()


def test_extreme_aspect_members_match_alone_bitwise():
    # 2^20 x 3 (4298 strips of one short segment) and 3 x 2^20 (one strip
    # whose lanes wrap the three columns, cut into many segments) in one pool
    # with its initial shape, 13 steps; bitwise equal to their own runs with
    # the default launches.
    import torch
    from paper_1107_4543_amd.pool import Pool
    s = SETS[1]
    pool = Pool(max_members=4, max_tiles=1 << 20)
    lats, twins = [], []
    for i, (nx, ny) in enumerate([(1 << 20, 3), (3, 1 << 20)]):
        lat, f = make(nx, ny, s, "f32", seed=80 + i, u0=(0.02, -0.01))
        pool.add(lat, 13)
        lats.append(lat)
        twins.append(twin(lat, f, s).step(13))
    pool.step(13)
    done = []
    while pool.members:
        done += pool.poll(wait=True)
    pool.close()
    assert len(done) == 2
    for lat, tw in zip(lats, twins):
        assert lat.t == 13 and torch.equal(lat.populations(), tw.populations()), (lat.nx, lat.ny)
