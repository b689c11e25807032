"""Serving with continuous batching: every job completes with exactly the
state it reaches when served alone (plain, one job at a time) -- compared
value by value for every job --, the served jobs agree with the FP64 oracle
within each storage type's tolerance, the HBM budget is never exceeded, and
jobs that can never fit are rejected."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs

pytestmark = pytest.mark.gpu


def small_trace(seed, n, rate, storages=("f32", "f16"), side_range=(48, 300), steps_range=(20, 400)):
    from paper_1107_4543_amd import stability
    return lbm_inputs.serving_trace(seed, rate, n, side_range=side_range, steps_range=steps_range,
                                    accept=stability.stable, storages=storages)


@pytest.mark.parametrize("policy", ["aged", "sjf", "fifo"])
def test_served_jobs_equal_plain_runs_and_respect_the_budget(policy):
    from paper_1107_4543_amd.serve import Server, footprint, run_plain
    trace = small_trace(11, 14, rate=400.0, storages=("f32", "f16", "bf16", "f64"))
    budget = 3 * max(footprint(s) for s in trace)          # at most ~3 jobs at once
    srv = Server(budget, max_members=8, chunk_ms=2.0, policy=policy, keep="state")
    served = {r.tag: r for r in srv.run(trace)}
    # FP16/BF16 jobs run in a pool of their own (six steps per launch)
    assert srv.half_pool is srv.pools[-1] and srv.half_pool.shape["steps_per_launch"] == 6
    srv.close()
    assert srv.peak_used <= budget and srv.peak_members >= 2
    assert sorted(served) == [s.tag for s in trace] and not srv.rejected
    plain = {r.tag: r for r in run_plain(trace, keep="state")}
    specs = {s.tag: s for s in trace}
    for tag, r in served.items():
        p = plain[tag]
        assert r.status == 0 and p.status == 0
        assert r.digest[0] == p.digest[0] == specs[tag].steps            # step count
        assert tuple(r.state.shape) == (9, specs[tag].ny, specs[tag].nx)
        assert torch.equal(r.state, p.state), tag                        # every stored value, bitwise
        assert r.diag == p.diag, tag
        assert r.done >= r.admitted >= r.arrival


def test_served_digests_equal_plain_digests():
    # the on-device digest that the serving benchmark compares
    from paper_1107_4543_amd.serve import Server, run_plain
    trace = small_trace(21, 10, rate=300.0)
    srv = Server(1 << 34, max_members=8, chunk_ms=2.0, keep="digest")
    served = {r.tag: r.digest for r in srv.run(trace)}
    srv.close()
    plain = {r.tag: r.digest for r in run_plain(trace, keep="digest")}
    assert served == plain
    assert len(set(served.values())) == len(trace)                       # distinct jobs, distinct digests


def test_lone_jobs_run_alone_join_the_pool_and_equal_plain_runs():
    # A long job starts on an empty server and advances alone with its own
    # launches; a second job arrives while it runs, so the first joins the
    # pool with the steps it has left; a third arrives long after both and
    # runs alone to the end.  Every final state equals its plain run's.
    import dataclasses
    from paper_1107_4543_amd.serve import Server, run_plain
    base = small_trace(41, 3, rate=100.0, storages=("f32", "f16", "f32"))
    trace = [dataclasses.replace(base[0], nx=512, ny=512, steps=5003, arrival=0.0, tag=0),
             dataclasses.replace(base[1], nx=200, ny=136, steps=777, arrival=0.005, tag=1),
             dataclasses.replace(base[2], nx=300, ny=260, steps=401, arrival=0.4, tag=2)]
    srv = Server(1 << 34, max_members=8, chunk_ms=2.0, keep="state")
    served = {r.tag: r for r in srv.run(trace)}
    srv.close()
    assert srv.solo_started == 2 and srv.solo_joined == 1, (srv.solo_started, srv.solo_joined)
    off = Server(1 << 34, max_members=8, chunk_ms=2.0, keep="state", solo=False)
    pooled = {r.tag: r for r in off.run(trace)}
    off.close()
    assert off.solo_started == 0
    # the 512^2 job counted as large: it keeps its own launches while the
    # second job runs in the pool beside it
    big = Server(1 << 34, max_members=8, chunk_ms=2.0, keep="state", solo_cells=1 << 18)
    beside = {r.tag: r for r in big.run(trace)}
    big.close()
    assert big.solo_started == 2 and big.solo_joined == 0, (big.solo_started, big.solo_joined)
    plain = {r.tag: r for r in run_plain(trace, keep="state")}
    for s in trace:
        assert served[s.tag].digest[0] == plain[s.tag].digest[0] == s.steps
        assert torch.equal(served[s.tag].state, plain[s.tag].state), s.tag
        assert torch.equal(pooled[s.tag].state, plain[s.tag].state), s.tag
        assert torch.equal(beside[s.tag].state, plain[s.tag].state), s.tag
        assert served[s.tag].diag == plain[s.tag].diag


def test_small_jobs_advance_at_their_own_pace_beside_large_ones():
    # A 2048^2 job starts alone; a 128^2 job with as many steps arrives while
    # it runs.  In pools by size class (2^18 and 2^21 cells) the small job
    # takes its steps in chunks of its own and finishes first; in one shared
    # pool (the default) every member advances by the same steps per chunk,
    # so it finishes with the large one.  Both equal plain runs bitwise.
    import dataclasses
    from paper_1107_4543_amd.serve import Server, run_plain
    base = small_trace(43, 2, rate=100.0, storages=("f32", "f32"))
    trace = [dataclasses.replace(base[0], nx=2048, ny=2048, steps=3000, arrival=0.0, tag=0),
             dataclasses.replace(base[1], nx=128, ny=128, steps=3000, arrival=0.004, tag=1)]
    srv = Server(1 << 34, max_members=8, keep="state", size_classes=(1 << 18, 1 << 21), half_pool=False)
    served = {r.tag: r for r in srv.run(trace)}
    srv.close()
    assert len(srv.pools) == 3 and srv.solo_joined == 1
    assert served[1].done < served[0].done, (served[1].done, served[0].done)
    one = Server(1 << 34, max_members=8, keep="state", half_pool=False)
    shared = {r.tag: r for r in one.run(trace)}
    one.close()
    assert len(one.pools) == 1
    plain = {r.tag: r for r in run_plain(trace, keep="state")}
    for s in trace:
        assert torch.equal(served[s.tag].state, plain[s.tag].state), s.tag
        assert torch.equal(shared[s.tag].state, plain[s.tag].state), s.tag


def _oracle_fields(spec):
    import oracle
    from oracle import linear
    relax = spec.relax
    s_nu = relax["s_nu"] if "s_nu" in relax else float(linear.s_from_nu(relax["nu"]))
    rates = [relax["s_e"], relax["s_eps"], relax["s_q"], s_nu]
    rho, ux, uy = spec.fields()
    f = oracle.run(oracle.init(rho, ux, uy), rates, spec.steps)
    r_or, u_or, v_or = oracle.moments(f)
    A = float(np.max(np.abs(rho - 1.0)))
    # velocity scale: the largest |u| of the input or of the oracle's result
    # (a pulse starts at rest)
    Au = max(float(np.max(np.abs(a))) for a in (ux, uy, u_or, v_or))
    return (r_or, u_or, v_or), A, Au


def test_served_jobs_match_the_oracle():
    # Served jobs (in the mix) against the FP64 oracle run of the same job:
    # FP64 storage to 1e-12 of the field, FP32 to 1e-5 of the fluctuation
    # amplitude, 16-bit storage within 3 u sqrt(steps) A (u the unit roundoff
    # of the stored type).  These jobs are short enough to finish alone
    # between arrivals, so the lone-job path is off: every job runs in the
    # pool's batched kernels (the lone path runs the plain launches, which the
    # parity tests check against the oracle).
    from paper_1107_4543_amd.serve import Server
    trace = small_trace(31, 12, rate=500.0, storages=("f64", "f32", "f16", "bf16"), side_range=(24, 96),
                        steps_range=(20, 300))
    assert {s.storage for s in trace} == {"f64", "f32", "f16", "bf16"}
    srv = Server(1 << 34, max_members=12, chunk_ms=2.0, keep="fields", solo=False)
    served = {r.tag: r for r in srv.run(trace)}
    srv.close()
    assert srv.peak_members >= 2
    unit = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
    for spec in trace:
        (r_or, u_or, v_or), A, Au = _oracle_fields(spec)
        rho, ux, uy = served[spec.tag].fields
        err_r = float(np.max(np.abs(rho - r_or)))
        err_u = max(float(np.max(np.abs(ux - u_or))), float(np.max(np.abs(uy - v_or))))
        if spec.storage == "f64":
            assert err_r <= 1e-12 * float(np.max(np.abs(r_or))), (spec.tag, err_r)
            assert err_u <= 1e-12 * float(np.max(np.abs(r_or))), (spec.tag, err_u)
        elif spec.storage == "f32":
            assert err_r <= 1e-5 * A, (spec.tag, err_r / A)
            assert err_u <= 1e-5 * Au, (spec.tag, err_u / Au)
        else:
            bound = 3 * unit[spec.storage] * math.sqrt(spec.steps) * A
            assert err_r <= bound, (spec.tag, spec.storage, err_r / A)


def test_jobs_larger_than_the_budget_are_rejected():
    from paper_1107_4543_amd.serve import Server, footprint
    trace = small_trace(12, 6, rate=1000.0)
    big = max(trace, key=footprint)
    budget = footprint(big) - 1
    srv = Server(budget, max_members=4, chunk_ms=2.0)
    done = srv.run(trace)
    srv.close()
    assert big.tag in srv.rejected
    assert len(done) + len(srv.rejected) == len(trace)
