"""Serving with continuous batching: every job completes with exactly the
result it gets when served alone (plain, one job at a time), the HBM budget is
never exceeded, and jobs that can never fit are rejected."""
import pytest

import lbm_inputs

pytestmark = pytest.mark.gpu


def small_trace(seed, n, rate):
    from paper_1107_4543_amd import stability
    return lbm_inputs.serving_trace(seed, rate, n, side_range=(48, 300), steps_range=(20, 400),
                                    accept=stability.stable)


def test_served_jobs_equal_plain_runs_and_respect_the_budget():
    from paper_1107_4543_amd.serve import Server, footprint, run_plain
    trace = small_trace(11, 14, rate=400.0)
    budget = 3 * max(footprint(s) for s in trace)          # at most ~3 jobs at once
    srv = Server(budget, max_members=8, chunk_ms=2.0)
    served = {r.tag: r for r in srv.run(trace)}
    srv.close()
    assert srv.peak_used <= budget and srv.peak_members >= 2
    assert sorted(served) == [s.tag for s in trace] and not srv.rejected
    plain = {r.tag: r for r in run_plain(trace)}
    for tag, r in served.items():
        assert r.status == 0
        assert r.diag == plain[tag].diag, tag              # bit-identical FP64 sums
        assert r.done >= r.admitted >= r.arrival


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
