"""Admission policy of the serving loop (host logic, no GPU).

The server admits queued jobs in the order ``order_queue`` gives, and a head
that does not fit blocks the jobs behind it.  Under a sustained stream of
small jobs that keeps the cell cap nearly full, shortest-job-first keeps
putting new small jobs ahead of a large one, so the large job waits until
the stream ends; with ageing ("aged", the server's default) a job that has
waited a fixed time plus a multiple of its estimated service time goes first, so the
large job reaches the head, blocks the stream until enough cells drain, and
is admitted after a bounded wait that does not depend on how long the
stream lasts.
"""
import importlib.util
import os
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _serve_module():
    # serve.py's policy functions need no GPU; load it with its package
    pytest.importorskip("torch")
    from paper_1107_4543_amd import serve
    return serve


def job(tag, arrival, cells, steps):
    return types.SimpleNamespace(tag=tag, arrival=arrival, nx=cells, ny=1, steps=steps)


def simulate(policy, jobs, cap_cells, lups_per_job):
    """Event-free time-stepped model of the server's admission: each admitted
    job runs at lups_per_job lattice updates per second (the cap is sized so
    the GPU serves every admitted job at full speed), the queue is re-ordered
    by policy before each admission round, the head is admitted while it fits
    under cap_cells, and a head that does not fit stops the round.  Returns
    {tag: admission time}."""
    serve = _serve_module()
    dt = 1e-3
    pending = sorted(jobs, key=lambda j: j.arrival)
    queue, active, admitted = [], [], {}
    t = 0.0
    while pending or queue or active:
        while pending and pending[0].arrival <= t:
            queue.append(pending.pop(0))
        queue = serve.order_queue(queue, policy, t)
        used = sum(j.nx * j.ny for j, _ in active)
        while queue and used + queue[0].nx * queue[0].ny <= cap_cells:
            j = queue.pop(0)
            admitted[j.tag] = t
            active.append((j, t + j.nx * j.ny * j.steps / lups_per_job))
            used += j.nx * j.ny
        t += dt
        active = [(j, end) for j, end in active if end > t]
    return admitted


def stream_with_large_job(burst_s=20.0):
    # cap 100 units; small jobs of 10 units lasting 1 s arrive every 0.125 s
    # (8 active: never 60 units free while they are admitted first); one
    # large job of 60 units lasting 4 s arrives at t = 0.5.  Jobs run at the
    # rate the policy assumes, so estimated service times are the true ones.
    serve = _serve_module()
    unit = 1000
    lups = serve.SERVICE_LUPS_ESTIMATE
    small_steps = int(lups * 1.0 / (10 * unit))
    jobs = [job(i, 0.125 * i, 10 * unit, small_steps) for i in range(int(burst_s / 0.125))]
    jobs.append(job(-1, 0.5, 60 * unit, int(lups * 4.0 / (60 * unit))))
    return jobs, 100 * unit, lups


def test_order_queue_policies():
    serve = _serve_module()
    a = job(1, 0.0, 1000, 10 ** 9)      # large (4 s at the assumed rate), oldest
    b = job(2, 1.0, 10, 100)            # small
    c = job(3, 1.5, 50, 100)
    assert serve.service_estimate(a) == pytest.approx(4.0)
    assert [j.tag for j in serve.order_queue([c, b, a], "fifo", 1.5)] == [1, 2, 3]
    assert [j.tag for j in serve.order_queue([a, c, b], "sjf", 1.5)] == [2, 3, 1]
    # nobody aged yet: shortest first
    assert not any(serve.is_aged(j, 1.5) for j in (a, b, c))
    assert [j.tag for j in serve.order_queue([a, c, b], "aged", 1.5)] == [2, 3, 1]
    # small jobs age after AGE_FIXED_S (their service is negligible), and
    # aged jobs go in arrival order ahead of younger ones
    t_small = 1.5 + serve.AGE_FIXED_S + 1e-6
    assert serve.is_aged(b, t_small) and serve.is_aged(c, t_small) and not serve.is_aged(a, t_small)
    assert [j.tag for j in serve.order_queue([a, c, b], "aged", t_small)] == [2, 3, 1]
    # once the large job has waited AGE_FIXED_S + AGE_FACTOR x 4 s it goes first
    t_old = serve.AGE_FIXED_S + serve.AGE_FACTOR * 4.0 + 1e-6
    assert serve.is_aged(a, t_old)
    d = job(4, t_old, 10, 100)          # just arrived: not aged, smallest
    assert [j.tag for j in serve.order_queue([d, c, b, a], "aged", t_old)] == [1, 2, 3, 4]
    with pytest.raises(ValueError):
        serve.order_queue([a], "lifo", 0.0)


def test_sjf_starves_the_large_job_and_ageing_bounds_its_wait():
    serve = _serve_module()
    burst = 40.0
    jobs, cap, lups = stream_with_large_job(burst)
    sjf = simulate("sjf", jobs, cap, lups)
    aged = simulate("aged", jobs, cap, lups)
    fifo = simulate("fifo", jobs, cap, lups)
    wait = {k: v[-1] - 0.5 for k, v in (("sjf", sjf), ("aged", aged), ("fifo", fifo))}
    # shortest-job-first: admitted only after the stream of small jobs ends
    assert wait["sjf"] >= burst - 1.0
    # ageing: the large job ages after AGE_FIXED_S + AGE_FACTOR x 4 s, then
    # waits at most for the admitted small jobs (1 s each) to free its room
    bound = serve.AGE_FIXED_S + serve.AGE_FACTOR * 4.0 + 1.0 + 0.01
    assert wait["aged"] <= bound, wait
    # every small job is still served, each within a bounded wait
    small_waits = [aged[j.tag] - j.arrival for j in jobs if j.tag >= 0]
    assert len(small_waits) == len(jobs) - 1 and max(small_waits) <= 20.0
    assert wait["fifo"] <= 0.01                # arrival order admits it at once here


def test_aged_wait_bound_does_not_grow_with_the_burst():
    jobs30, cap, lups = stream_with_large_job(30.0)
    jobs60, _, _ = stream_with_large_job(60.0)
    w30 = simulate("aged", jobs30, cap, lups)[-1] - 0.5
    w60 = simulate("aged", jobs60, cap, lups)[-1] - 0.5
    assert abs(w60 - w30) <= 0.01


def test_chunks_are_whole_launches_of_about_chunk_ms():
    # a chunk is about chunk_ms of device work at the assumed update rate, at
    # most 1024 steps, and a whole number of T-step launches when it is at
    # least one launch long (a lone job or a pool advances in chunks of it)
    serve = _serve_module()
    srv = types.SimpleNamespace(chunk_ms=5.0)
    for T in (1, 6, 7):
        for cells in (128 * 128, 724 * 724, 2048 * 2048, 4096 * 4096, 1 << 25):
            n = serve.Server._chunk(srv, cells, T)
            assert 1 <= n <= 1024
            if n >= T:
                assert n % T == 0, (T, cells, n)
            # within one launch of the target duration, or at the step cap
            want = 5.0 / max(cells / serve.SERVICE_LUPS_ESTIMATE * 1e3, 0.004)
            assert n <= want and (n + T > min(want, 1024) or n == 1024 - 1024 % T), (T, cells, n, want)
    # a 4096^2 lattice: ~5 ms at 2.5e11 updates/s is 74 steps, 70 in seven-step launches
    assert serve.Server._chunk(srv, 4096 * 4096, 7) == 70
    # small lattices are bounded by the step cap
    assert serve.Server._chunk(srv, 128 * 128, 7) == 1022
