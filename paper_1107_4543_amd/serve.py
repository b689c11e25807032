"""Serving D2Q9 MRT simulation jobs on one GPU with continuous batching.

A job is a lattice (size, relaxation rates, storage type, initial fields) and
a number of steps.  ``Server.run`` replays a trace of jobs in real time:

* jobs whose arrival time has passed wait in a queue, ordered by the
  admission policy: shortest job first with ageing ("aged", the default:
  least cells x steps first, but a job that has waited a fixed second plus
  four times its estimated service time goes ahead of all younger jobs, so
  no job starves), plain shortest job first ("sjf") or arrival order
  ("fifo");
* the head of the queue is admitted as soon as its device footprint fits in
  the HBM budget, the pool has a free member slot and the cells being
  advanced stay under a cap: its workspace is allocated, its fields are
  generated on the device and it joins the pool (its state stays on the
  device for its whole life); a head that does not fit blocks the jobs
  behind it (no backfilling), which bounds its wait;
* the pool advances all admitted jobs together, one chunk of about
  ``chunk_ms`` of device work at a time (persistent batched launches,
  recorded step loop), with at most two rounds of chunks in flight so that
  admissions and completions are handled between them; jobs with 16-bit
  storage have a pool of their own (``half_pool``), with the launch shape
  that suits them, whose chunks run beside the main pool's.  Every member
  of a pool advances by the same number of steps per chunk, so a small
  lattice beside a large one moves at the large one's pace (a 128^2 job
  beside a 4096^2 one: ~70 steps per 5 ms chunk instead of over a
  thousand).  With
  ``size_classes`` the jobs go to one pool per size class instead, whose
  chunks take turns on one stream: small jobs then move at their own pace,
  but the pools no longer share launches;
  a job admitted to an empty server with nothing queued behind it advances
  alone with its own lattice's default launches (``solo``), and joins the
  pool with its remaining steps as soon as a second job is admitted (every
  launch shape gives the same values, so the result does not depend on
  when, or whether, it joins);
* a job leaves the pool after exactly its own number of steps; its result
  is read and its memory returned to the budget: the FP64 mass/momentum
  diagnostics, and (``keep``) a digest of its raw final state, or the raw
  state itself, or its FP64 density and velocity fields.

``run_plain`` serves the same trace one job at a time in arrival order with
each lattice's own default launches, for comparison.  Both paths use the
same per-cell arithmetic, so every job's final state is bit-identical in the
two; the digests (or states) let a caller check that for every job.
"""
import collections
import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import torch

from . import _lib
from .lattice import Lattice
from .pool import Pool
from . import stability

STORE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


@dataclass
class JobResult:
    tag: int
    arrival: float
    admitted: float
    done: float
    nx: int
    ny: int
    steps: int
    storage: str
    diag: List[float] = field(default_factory=list)
    status: int = 0
    digest: Optional[tuple] = None       # state_digest of the final raw state
    state: Optional[object] = None       # final raw state bytes (host uint8 tensor)
    fields: Optional[tuple] = None       # final (rho, ux, uy), host float64 arrays

    @property
    def latency(self):
        return self.done - self.arrival


def footprint(spec):
    """Device bytes a job holds while admitted: its workspace plus its three
    FP64 initial fields."""
    d = _lib.lbm_desc()
    d.nx, d.ny = spec.nx, spec.ny
    d.storage = _lib.STORAGE[spec.storage]
    d.compute = _lib.LBM_COMPUTE_F64 if spec.storage == "f64" else _lib.LBM_COMPUTE_F32
    d.s_e, d.s_eps, d.s_q, d.s_nu = stability.rates(spec.relax)
    d.rho0, d.u0x, d.u0y = 1.0, 0.0, 0.0
    d.scale_exp = _lib.LBM_SCALE_AUTO
    d.flags = 0
    return _lib.lbm_workspace_bytes(d) + 24 * spec.nx * spec.ny


def _new_lattice(spec, device, stream=None):
    """Allocates, generates the initial fields and initialises on `stream`."""
    stream = stream if stream is not None else torch.cuda.current_stream(device)
    with torch.cuda.stream(stream):
        lat = Lattice(spec.nx, spec.ny, *stability.rates(spec.relax), storage=spec.storage, device=device,
                      stream=stream)
        lat.init(*spec.fields_torch(device))
    return lat


# odd 64-bit multipliers of the position-weighted digest
_DIGEST_MUL, _DIGEST_ADD = 0x9E3779B97F4A7C15 - (1 << 64), 0x632BE59BD9B4E019


_RAW_INT = {"f64": torch.int64, "f32": torch.int32, "f16": torch.int16, "bf16": torch.int16}


def raw_state(lat):
    """The lattice's raw stored populations as a [9, ny, nx] integer device
    tensor (the storage type's bit patterns; the row padding that the
    library's layout carries beyond nx is dropped), ordered on the
    lattice's stream, and the step count t."""
    buf, t = lat.save_state()
    E = STORE_BYTES[lat.storage]
    pitch = buf.numel() // (9 * lat.ny * E)
    with torch.cuda.stream(lat.stream):
        raw = buf.view(_RAW_INT[lat.storage]).view(9, lat.ny, pitch)[:, :, :lat.nx]
    return raw, t


def state_digest(lat):
    """Digest of a lattice's raw state, computed on the device: the step
    count and the wrapping int64 sums of the stored values' bit patterns and
    of each pattern times an odd position-dependent multiplier.  Two states
    with equal digests are equal except with negligible probability; any one
    changed value changes both sums."""
    raw, t = raw_state(lat)
    with torch.cuda.stream(lat.stream):
        words = raw.reshape(-1).to(torch.int64)
        pos = torch.arange(words.numel(), dtype=torch.int64, device=words.device)
        weights = pos * _DIGEST_MUL + _DIGEST_ADD
        weights |= 1
        d = torch.stack([words.sum(), (words * weights).sum()])
        host = d.cpu()                  # ordered after the sums on the lattice's stream
    return (t,) + tuple(int(v) for v in host)


def _keep_result(lat, keep):
    """What a finished job hands back besides its diagnostics."""
    if keep == "digest":
        return {"digest": state_digest(lat)}
    if keep == "state":
        raw, t = raw_state(lat)
        with torch.cuda.stream(lat.stream):
            host = raw.cpu()
        return {"digest": (t,), "state": host}
    if keep == "fields":
        with torch.cuda.stream(lat.stream):
            return {"fields": tuple(a.cpu().numpy() for a in lat.moments())}
    if keep in (None, "none"):
        return {}
    raise ValueError(f"keep must be None, 'digest', 'state' or 'fields', not {keep!r}")


def percentile(xs, q):
    if not xs:
        return float("nan")
    s = sorted(xs)
    k = (len(s) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


# lattice updates per second the admission policy assumes for one job's
# estimated service time
SERVICE_LUPS_ESTIMATE = 2.5e11
# a queued job is "aged" once it has waited AGE_FIXED_S + AGE_FACTOR times its
# estimated service time: late enough that a lightly loaded server never
# reorders (it then admits shortest first), soon enough to bound every wait
AGE_FIXED_S = 1.0
AGE_FACTOR = 4.0


def service_estimate(spec):
    """Seconds the job would take alone at SERVICE_LUPS_ESTIMATE."""
    return spec.nx * spec.ny * spec.steps / SERVICE_LUPS_ESTIMATE


def is_aged(spec, now):
    return now - spec.arrival >= AGE_FIXED_S + AGE_FACTOR * service_estimate(spec)


def order_queue(queue, policy, now):
    """The queue in admission order for `policy` at time `now` (seconds of
    the trace's clock): "fifo" by arrival; "sjf" by work (cells x steps);
    "aged" shortest job first, except that aged jobs (waited at least
    AGE_FIXED_S + AGE_FACTOR x their estimated service time) go first, in
    arrival order.  With the server's head blocking, an aged job at the head
    holds back every job behind it until it fits, so its wait is bounded by
    its ageing time plus the time the admitted jobs take to free its room."""
    if policy == "fifo":
        return sorted(queue, key=lambda s: (s.arrival, s.tag))
    if policy == "sjf":
        return sorted(queue, key=lambda s: (s.nx * s.ny * s.steps, s.arrival, s.tag))
    if policy == "aged":
        return sorted(queue, key=lambda s: (0, s.arrival, s.tag) if is_aged(s, now)
                      else (1, s.nx * s.ny * s.steps, s.arrival, s.tag))
    raise ValueError(f"policy must be 'aged', 'sjf' or 'fifo', not {policy!r}")


_SIDE_STREAMS = {}


def _side_stream(device, name="side"):
    """One stream per device and purpose, shared by every server of the
    process (default priority)."""
    key = (torch.device(device).index or 0, name)
    if key not in _SIDE_STREAMS:
        _SIDE_STREAMS[key] = torch.cuda.Stream(torch.device(device))
    return _SIDE_STREAMS[key]


class Server:
    """policy: "aged" (default) admits the queued job with the least work
    (cells x steps) first unless a job has aged (see order_queue), "sjf" the
    one with the least work, "fifo" in arrival order.  max_active_cells caps
    the cells being advanced at once (a job larger than the cap runs when
    nothing else does), in addition to the HBM budget and the member slots.
    Against 2^25, a cap of 2^24 (one 4096^2 lattice) measured a 30-45 %
    lower median under load, but 3-10 % less aggregate throughput and on
    one trace an 11-17 % higher p99 at 100-300 jobs/s.  keep:
    what each JobResult carries besides the diagnostics (None, "digest",
    "state" or "fields").  solo: a job admitted to an empty server with
    nothing queued advances with its lattice's own default launches until a
    second job is admitted (the pool's batched kernels pay a table lookup
    and a launch shape shared by every member; one job alone runs faster
    with the shape chosen for its lattice).  solo_cells: jobs of at least
    this many cells also keep their own launches (on a stream of their own,
    beside the pool's) while no job waits in the queue, and join the pool
    once one does; None (the default) leaves them to the pool.  Measured: a
    lower median and mean at light load, a higher p99 (a large job beside a
    concurrent pool is slowed more than in the pool, whose small members
    barely slow it).  half_pool: jobs with 16-bit storage go to a pool of
    their own, with six steps per launch and loads one row ahead (their
    single-lattice shape; the main pool's seven steps suit FP32), on a
    stream of its own beside the main pool's; measured a 10-25 % lower
    median under load, p99 and aggregate within a few percent either way.
    size_classes: the cell counts
    that separate pools by lattice size (ascending; the default () puts
    every job in one pool, which measured the higher aggregate rate and the
    lower mean latency under load; classes gave the lower median)."""

    def __init__(self, hbm_budget_bytes, max_members=256, max_tiles=1 << 20, chunk_ms=5.0,
                 device="cuda:0", screen=False, policy="aged", max_active_cells=1 << 25,
                 tile_cells=512, keep=None, solo=True, size_classes=(), solo_cells=None, half_pool=True):
        self.device = torch.device(device)
        self.budget = int(hbm_budget_bytes)
        if list(size_classes) != sorted(set(size_classes)) or any(c <= 0 for c in size_classes):
            raise ValueError(f"size_classes must be ascending positive cell counts, not {size_classes!r}")
        self.size_classes = tuple(int(c) for c in size_classes)
        self.pools = []
        for _ in range(len(self.size_classes) + 1):
            pool = Pool(max_members=max_members, max_tiles=max_tiles, device=self.device,
                        stream=self.pools[0].stream if self.pools else None)
            pool.set_shape(tile_cells=tile_cells, block=512, grid=4096, graph_steps=256)
            self.pools.append(pool)
        self.half_pool = None
        if half_pool:
            # 16-bit storage in a pool of its own with the shape that suits it
            # (six steps per launch, loads one row ahead), on its own stream
            self.half_pool = Pool(max_members=max_members, max_tiles=max_tiles, device=self.device,
                                  stream=_side_stream(self.device, "half"))
            self.half_pool.set_shape(tile_cells=tile_cells, block=512, grid=4096, graph_steps=256,
                                     steps_per_launch=6, flags=34)
            self.pools.append(self.half_pool)
        self.steps_per_launch = self.pools[0].shape["steps_per_launch"]
        self._spl = {id(p): p.shape["steps_per_launch"] for p in self.pools}
        self.max_members = max_members
        self.chunk_ms = chunk_ms
        if policy not in ("aged", "sjf", "fifo"):
            raise ValueError(f"policy must be 'aged', 'sjf' or 'fifo', not {policy!r}")
        self.policy = policy
        self.keep = keep
        self.max_active_cells = max_active_cells
        self.solo = solo
        self.solo_cells = solo_cells
        self.screen = screen
        self.used = 0
        self.peak_used = 0
        self.peak_members = 0
        self.rejected = []
        self.solo_started = 0                        # jobs that began alone
        self.solo_joined = 0                         # ... and joined the pool with steps left
        # Jobs are initialised and read back on a side stream: a finished
        # job's readback then waits for its own last chunk only, not for the
        # chunks enqueued after it on the pool's stream.  One such stream per
        # device serves every server of the process: torch's caching
        # allocator reuses a freed block only on the stream it was allocated
        # on, so a stream per server would keep every earlier server's job
        # memory reserved.
        self.side = _side_stream(self.device)
        self.solo_stream = _side_stream(self.device, "solo")

    def _pool_of(self, spec):
        if self.half_pool is not None and spec.storage in ("f16", "bf16"):
            return self.half_pool
        cells = spec.nx * spec.ny
        return self.pools[sum(1 for c in self.size_classes if cells >= c)]

    def _chunk_steps(self, active_cells, pool=None):
        # about chunk_ms of device work at the pool's update rate (short steps
        # are bounded below by launch cost), in whole T-step launches: a count
        # that is not a multiple of T ends every chunk in one-step launches
        return self._chunk(active_cells, self._spl[id(pool)] if pool is not None else self.steps_per_launch)

    def _chunk(self, cells, spl):
        est_ms = max(cells / SERVICE_LUPS_ESTIMATE * 1e3, 0.004)
        n = max(1, min(1024, int(self.chunk_ms / est_ms)))
        return n - n % spl if n >= spl else n

    def run(self, trace) -> List[JobResult]:
        pending = collections.deque(sorted(trace, key=lambda s: s.arrival))
        queue = collections.deque()
        active = {}                                  # id(lattice) -> (spec, admitted, bytes, lattice)
        inflight = collections.deque()               # rounds: the events of one round of chunks
        results = []
        # jobs advancing outside the pools with their own launches, by
        # id(lattice): [lattice, steps not yet enqueued, event after the
        # last step (once all are enqueued), spec, large (joins a pool only
        # when jobs wait in the queue; else when any other job is pooled)]
        solos = {}
        t0 = time.perf_counter()
        while pending or queue or active:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # admission by HBM budget, member slots and the active-cells cap
            if len(queue) > 1:
                queue = collections.deque(order_queue(queue, self.policy, now))
            while queue:
                spec = queue[0]
                need = footprint(spec)
                if need > self.budget or (self.screen and not stability.stable(spec.relax)):
                    self.rejected.append(queue.popleft().tag)
                    continue
                active_cells = sum(a[0].nx * a[0].ny for a in active.values())
                if (self.used + need > self.budget or len(active) >= self.max_members
                        or (active and active_cells + spec.nx * spec.ny > self.max_active_cells)):
                    break
                big = self.solo_cells is not None and spec.nx * spec.ny >= self.solo_cells
                backlog = len(queue) > 1                 # others wait behind this job
                alone = self.solo and not active and not backlog
                own = alone or (big and not backlog)
                lat = _new_lattice(spec, self.device, self.solo_stream if big and own else self.side)
                if own:
                    solos[id(lat)] = [lat, spec.steps, None, spec, big]
                    self.solo_started += 1
                else:
                    for k, e in list(solos.items()):
                        if e[1] > 0 and (not e[4] or backlog):
                            # a second job: the lone one joins its pool with
                            # the steps it has left (the pool waits for its
                            # queued ones); with the pool's tile table full it
                            # keeps its own launches
                            try:
                                self._pool_of(e[3]).add(e[0], e[1])
                            except _lib.LbmError as err:
                                if err.status != _lib.LBM_E_NOMEM:
                                    raise
                                continue
                            del solos[k]
                            self.solo_joined += 1
                    try:
                        self._pool_of(spec).add(lat, spec.steps)
                    except _lib.LbmError as e:
                        if e.status != _lib.LBM_E_NOMEM or not active:
                            raise
                        lat.close()                  # tile table full: retry when a job leaves
                        break
                queue.popleft()
                active[id(lat)] = (spec, time.perf_counter() - t0, need, lat)
                self.used += need
                self.peak_used = max(self.peak_used, self.used)
                self.peak_members = max(self.peak_members, len(active))
            streams = []
            for pool in self.pools:
                running = [a for a in active.values()
                           if id(a[3]) not in solos and self._pool_of(a[0]) is pool and pool.remaining(a[3]) > 0]
                if running:
                    pool.step(self._chunk_steps(sum(a[0].nx * a[0].ny for a in running), pool))
                    if all(pool.stream is not s for s in streams):
                        streams.append(pool.stream)
            events = []
            for s in streams:
                ev = torch.cuda.Event()
                ev.record(s)
                events.append(ev)
            for e in solos.values():
                if e[2] is not None:
                    continue
                lat = e[0]
                n = min(e[1], self._chunk(lat.nx * lat.ny, lat.steps_per_launch))
                if n > 0:
                    lat.step(n)
                    e[1] -= n
                ev = torch.cuda.Event()
                ev.record(lat.stream)
                events.append(ev)
                if e[1] == 0:
                    e[2] = ev
            enqueued = bool(events)
            if events:
                inflight.append(events)
            while len(inflight) > 2:
                for ev in inflight.popleft():
                    ev.synchronize()
            finished = []
            for pool in self.pools:
                finished += pool.poll()
            for k, e in list(solos.items()):
                if e[2] is not None and e[2].query():
                    finished.append(e[0])
                    del solos[k]
            if not enqueued and not finished and inflight:
                # every admitted job has all its steps enqueued: wait for the
                # oldest round in flight, after which the next may be done
                for ev in inflight.popleft():
                    ev.synchronize()
            for lat in finished:
                spec, admitted, need, _ = active.pop(id(lat))
                status, diag = lat.diagnostics()
                kept = _keep_result(lat, self.keep)
                done = time.perf_counter() - t0
                results.append(JobResult(spec.tag, spec.arrival, admitted, done, spec.nx, spec.ny, spec.steps,
                                         spec.storage, diag, status, **kept))
                lat.close()
                self.used -= need
            if not active and not queue and pending:
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
        return results

    def close(self):
        for pool in self.pools:
            pool.close()


def run_plain(trace, device="cuda:0", keep=None) -> List[JobResult]:
    """One job at a time in arrival order, each with its lattice's default
    launch shape (several steps per launch from 2^19 cells, else one)."""
    results = []
    t0 = time.perf_counter()
    for spec in sorted(trace, key=lambda s: s.arrival):
        now = time.perf_counter() - t0
        if spec.arrival > now:
            time.sleep(spec.arrival - now)
        admitted = time.perf_counter() - t0
        lat = _new_lattice(spec, device)
        lat.step(spec.steps)
        status, diag = lat.diagnostics()
        kept = _keep_result(lat, keep)
        done = time.perf_counter() - t0
        results.append(JobResult(spec.tag, spec.arrival, admitted, done, spec.nx, spec.ny, spec.steps,
                                 spec.storage, diag, status, **kept))
        lat.close()
    return results


def summarize(results: List[JobResult]):
    lat = [r.latency for r in results]
    lups = sum(r.nx * r.ny * r.steps for r in results)
    span = max(r.done for r in results) - min(r.arrival for r in results) if results else float("nan")
    return {"jobs": len(results), "p50_s": round(percentile(lat, 50), 4), "p99_s": round(percentile(lat, 99), 4),
            "max_s": round(max(lat), 4) if lat else None,
            "mean_s": round(sum(lat) / max(1, len(lat)), 4), "makespan_s": round(span, 4),
            "aggregate_mlups": round(lups / span / 1e6, 1) if span > 0 else None,
            "nonfinite_jobs": sum(1 for r in results if r.status != 0)}
