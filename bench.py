"""Benchmark of the D2Q9 MRT lattice Boltzmann step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload waves4096]

Workload (default): 4096 x 4096 periodic lattice, FP32 deviation storage and
arithmetic, Table 5 group A relaxation rates, a plane acoustic wave
(k = 2 pi 8 / 4096 along x, amplitude 1e-4) plus a shear wave (u_y amplitude
1e-4) on a mean flow u_x = 0.1 c_s; the job is 2000 steps.  One "step" is one
collide-and-stream update of the whole lattice; the tuned launch shape may
advance several steps per kernel launch (temporal blocking in registers).
The inputs are resident in HBM before timing starts; the timed region is K
consecutive steps on the lattice's stream, bracketed by device
synchronisation and HIP events.

Prints one JSON line: MLUPS, the roofline of the step kernel over its
measured average launch duration -- for one step per launch the HBM bound
(algorithmic bytes 2 * 9 * sizeof(storage) per cell and launch against the
8 TB/s peak); for several steps per launch the vector-ALU bound (the
collision's 70 (FP32, FP64) or 71 (16-bit storage) algorithmic operations
per cell and step against the non-packed issue peak), with the HBM figures
beside it -- measured HBM traffic from the committed rocprofv3 counter
summary when it matches the current kernel source, and the FP64 CPU oracle
timed on a bounded sample of the same workload on the host cores.  Beside the
single lattice the line carries the batched workload (256 lattices advanced
together by the pool kernel against one at a time) and one served trace
(Poisson arrivals of simulation jobs, continuous batching against one job at
a time: latency percentiles, aggregate MLUPS and per-job digest equality).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "MLUPS & % HBM roofline (D2Q9 MRT, 1 GPU); served p50/p99 vs plain at equal error"
STORE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


KERNEL_SOURCES = ("lbm_device.hpp", "lbm_step_common.hpp", "lbm_kernels.hip", "lbm_multi_f32.hip",
                  "lbm_multi_f64.hip", "lbm_multi_f16.hip", "lbm_multi_bf16.hip")   # the files that define the device code


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1107_4543_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()


VALU_PEAK = 256 * 4 * 16 * 2.4e9      # VALU lane-instructions per second (non-packed)
# Arithmetic of one lattice update in the compute type: the folded
# collision's additions, multiplications and fused multiply-adds plus its
# reciprocal (the moment sums, equilibrium numerators, relaxation, M^T and
# the increment; the kernels' comments list them): 69 + 1 where the storage
# type is the compute type (FP32, FP64: the rest population's update is one
# multiply-add), 70 + 1 otherwise (16-bit storage, FP64 storage with FP32
# collide: the rest population's increment is formed, then added).
# Vector-ALU peaks in operations per second: one operation per lane and clock
# on 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz in FP32 (packed FP32 is not
# used), half that in FP64.
def alg_ops_per_lu(storage, compute):
    return 70 if storage == compute else 71


ALU_PEAK = {"f32": 256 * 4 * 16 * 2.4e9, "f64": 256 * 4 * 16 * 2.4e9 / 2}


def read_profile(workload, storage, launch):
    """Key/value lines of the committed counter summary for this kernel, or
    None when absent, taken on a different kernel source, or on another
    kernel (variant and flags select the kernel; the summary names the shape
    it was taken with)."""
    kernel = "step_multi" if launch["variant"] >= 8 else "step"
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{storage}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    shape = kv.get("launch", "").split(",")
    if len(shape) != 6 or int(shape[0]) != launch["variant"] or int(shape[5]) != launch["flags"]:
        return None
    return kv


def read_traffic(workload, storage, launch):
    """Measured HBM bytes per launch (see read_profile), or None."""
    kv = read_profile(workload, storage, launch)
    try:
        return float(kv["traffic_bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


# Launch shapes measured fastest for the 4096^2 wave workload on MI355X
# (variants 11, 12 and 13: five, six and seven steps per pass; flag 32: the
# workgroup-shared halo); the library's defaults for this lattice; --tune
# searches again.
DEFAULT_LAUNCH = {"f32": "13,64,4,92,1,32", "f16": "12,64,4,69,1,34", "bf16": "12,64,4,69,1,40",
                  "f64": "13,64,4,137,1,32"}


def build_waves4096(storage):
    import numpy as np
    import torch

    import lbm_inputs
    from paper_1107_4543_amd import Lattice
    w = lbm_inputs.WORKLOADS["waves4096"]
    s = lbm_inputs.PRESETS[w["relax"]]
    rates = [s["s_e"], s["s_eps"], s["s_q"], s["s_nu"]]
    nx, ny = w["nx"], w["ny"]
    rho, ux, uy = lbm_inputs.plane_waves(nx, 1, w["mode"], w["amplitude"], w["shear_amplitude"], w["u0x"])
    fields = [torch.from_numpy(np.broadcast_to(a, (ny, nx)).copy()).cuda() for a in (rho, ux, uy)]
    lat = Lattice(nx, ny, *rates, storage=storage, u0=(w["u0x"], 0.0), device="cuda:0")
    lat.init(*fields)
    del fields
    cfg = {"workload": "waves4096", "nx": nx, "ny": ny, "storage": storage,
           "relaxation": "Table 5 group A", "u0x": w["u0x"], "mode": w["mode"],
           "amplitude": w["amplitude"], "job_steps": w["steps"]}
    return lat, cfg, rates, (rho, ux, uy), w


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(rates, fields1, nx, ny, u0x, budget_s, budget_1t_s):
    """FP64 oracle (as it stands) on the full lattice for as many whole steps
    as fit in about budget_s seconds (at least one) with its default OpenMP
    threads, and for about budget_1t_s seconds on one thread."""
    import numpy as np

    import oracle
    rho, ux, uy = (np.ascontiguousarray(np.broadcast_to(a, (ny, nx))) for a in fields1)
    f = oracle.init(rho, ux, uy)
    del rho, ux, uy

    def timed(budget):
        nonlocal f
        steps, elapsed = 0, 0.0
        while elapsed < budget or steps == 0:
            t0 = time.perf_counter()
            f = oracle.run(f, rates, 1)
            elapsed += time.perf_counter() - t0
            steps += 1
        return steps, elapsed

    cores = oracle.threads()
    steps, elapsed = timed(budget_s)
    out = {"value": nx * ny * steps / elapsed / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"FP64 oracle (unfused collide then stream) on the full {nx}x{ny} lattice, "
                     f"{steps} step(s), {elapsed:.1f} s, {cores} OpenMP threads",
           "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count()}
    if budget_1t_s > 0:
        oracle.set_threads(1)
        try:
            steps1, elapsed1 = timed(budget_1t_s)
        finally:
            oracle.set_threads(cores)
        out["one_thread"] = {"value": nx * ny * steps1 / elapsed1 / 1e6, "unit": "MLUPS", "cores": 1,
                             "sample": f"same, {steps1} step(s), {elapsed1:.1f} s, 1 thread"}
    return out


def copy_probe(nbytes, reps):
    """Plain device-to-device copy of nbytes, reps times (the calibration
    kernel for the HBM byte counters and the achievable-bandwidth context)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    return {"bytes_per_copy": nbytes, "us_per_copy": round(us, 2),
            "GBps": round(2 * nbytes / (us * 1e-6) / 1e9, 1)}


def read_pool_traffic(shape):
    """Measured HBM bytes per T-step launch of the pool kernel on batch256
    from the committed counter summary, or None when absent, taken on a
    different kernel source or with a different T-step shape."""
    path = os.path.join(ROOT, "profiles", "traffic_pool_multi_f32_batch256.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    want = ",".join(str(shape[k]) for k in ("steps_per_launch", "seg_rows", "waves", "flags"))
    if kv.get("pool_multi_shape") != want:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def pool_roofline(T, cells, launches, ms, traffic=None, steps=None):
    """Roofline of the pool's step kernel over a timed pass of `steps` steps
    that each member (FP32 storage and collide) takes in `launches` launches:
    HBM for one step per launch, the vector ALU (algorithmic operations,
    FP32) for T > 1, counting the updates of the steps actually run."""
    ops_lu = alg_ops_per_lu("f32", "f32")
    us = 1e3 * ms / launches
    gbps = 72 * cells / (us * 1e-6) / 1e9
    hbm = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
           "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": traffic, "algorithmic_bytes_per_launch": 72 * cells}
    common = {"kernel": ("k_pool_multi (%d steps per launch, persistent, per storage class)" % T if T > 1
                         else "k_pool_step (persistent, per storage class)"),
              "steps_per_launch": T, "launches": launches, "avg_launch_us": round(us, 3)}
    if T == 1:
        return dict(hbm, **common)
    steps = launches * T if steps is None else steps
    ops = ops_lu * cells * steps
    tops = ops / (ms * 1e-3) / 1e12
    peak = ALU_PEAK["f32"] / 1e12
    return dict({"bound": "alu", "achieved": round(tops, 2), "peak": round(peak, 2), "unit": "T F32 ops/s",
                 "frac": round(tops / peak, 4), "traffic": traffic,
                 "algorithmic_ops_per_launch": round(ops / launches), "algorithmic_ops_timed": ops,
                 "ops_per_update": ops_lu, "hbm": hbm}, **common)


# Pool shape measured fastest for batch256 on MI355X (seven steps per launch,
# strip tasks of about 96 rows, one workgroup of 4 waves sharing its halo
# columns through LDS per task, a member's left-over columns in two-wave
# workgroups when they fit: flags 96).  The pool's initial shape differs
# only in flags 32 (left-over columns in a narrower four-wave strip), which
# is faster for the few large lattices of a lightly loaded pool.
DEFAULT_POOL_SHAPE = "256,512,4096,256,7,96,4,96"
POOL_SHAPE_KEYS = ["tile_cells", "block", "grid", "graph_steps", "steps_per_launch", "seg_rows", "waves", "flags"]


def parse_pool_shape(text):
    vals = [int(v) for v in text.split(",")]
    if len(vals) != len(POOL_SHAPE_KEYS):
        raise SystemExit("--pool-shape takes " + ",".join(POOL_SHAPE_KEYS))
    return dict(zip(POOL_SHAPE_KEYS, vals))


def pool_member_launches(shape, steps):
    """Launches each member takes for `steps` steps: replays the pool's
    chunking (loops of T 2^m steps, then the remaining r < T steps as one
    pass)."""
    T = shape["steps_per_launch"]
    member_launches, left = 0, steps
    while left > 0:
        lim = min(left, shape["graph_steps"])
        if T > 1 and lim >= T:
            kk = T
            while kk * 2 <= lim:
                kk *= 2
            member_launches += kk // T
        elif T > 1:
            kk = lim                    # one pass of the remaining steps (one step: one launch)
            member_launches += 1
        else:
            kk = 1
            while kk * 2 <= lim:
                kk *= 2
            member_launches += kk
        left -= kk
    return member_launches


def run_batch256(steps, pool_shape=None, sequential=True):
    """256 independent lattices (sides log-uniform in [64, 1024], sampled
    stable rates, one pulse each, FP32): `steps` steps of all of them in one
    pool (persistent launches of several steps each, recorded step loop;
    pool_shape fixed, or tuned when None), timed with HIP events on the
    pool's stream, against the same 256 lattices run one after another with
    each lattice's default launches.  Returns a dict of the measurements."""
    import torch

    import lbm_inputs
    from paper_1107_4543_amd import Lattice, stability
    from paper_1107_4543_amd.pool import Pool
    w = lbm_inputs.WORKLOADS["batch256"]
    draws = [0]

    def accept(relax):
        draws[0] += 1
        return stability.stable(relax)

    specs = lbm_inputs.batch_specs(w["seed"], w["count"], steps=steps, accept=accept)
    dev = "cuda:0"
    lats = [Lattice(sp.nx, sp.ny, *stability.rates(sp.relax), storage="f32", device=dev) for sp in specs]
    fields = [sp.fields_torch(dev) for sp in specs]
    cells = sum(sp.nx * sp.ny for sp in specs)

    def init_all():
        for lat, f in zip(lats, fields):
            lat.init(*f)

    pool = Pool(max_members=len(specs), max_tiles=1 << 18, device=dev)
    init_all()
    for lat in lats:
        pool.add(lat, steps)
    if pool_shape:
        pool.set_shape(**pool_shape)
        shape = pool.shape
    else:
        shape, _ = pool.tune(reps=3)
    pool.step(steps)                                  # untimed warm-up pass (records the graph)
    while pool.members:
        pool.poll(wait=True)
    init_all()
    for lat in lats:
        pool.add(lat, steps)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(pool.stream)
    pool.step(steps)
    e1.record(pool.stream)
    torch.cuda.synchronize()
    ms_batched = e0.elapsed_time(e1)
    while pool.members:
        pool.poll(wait=True)
    batched_rho = [lat.moments()[0] for lat in lats]

    ms_seq, equal = None, None
    if sequential:
        init_all()
        torch.cuda.synchronize()
        e0.record()
        for lat in lats:
            lat.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms_seq = e0.elapsed_time(e1)
        equal = all(torch.equal(r, lat.moments()[0]) for r, lat in zip(batched_rho, lats))
    pool.close()
    return {"ms_batched": ms_batched, "ms_seq": ms_seq, "equal": equal, "shape": shape, "cells": cells,
            "lattices": len(specs), "draws": draws[0], "seq_launch": lats[0].launch, "seed": w["seed"]}


def batch_summary(r, steps):
    """MLUPS, roofline and comparison figures of a run_batch256 result."""
    lups = r["cells"] * steps
    T = r["shape"]["steps_per_launch"]
    member_launches = pool_member_launches(r["shape"], steps)
    ms_seq = r["ms_seq"]
    return {
        "value": round(lups / (r["ms_batched"] / 1e3) / 1e6, 1), "unit": "MLUPS", "steps": steps,
        "ms_per_step": round(r["ms_batched"] / steps, 5),
        "roofline": pool_roofline(T, r["cells"], member_launches, r["ms_batched"], read_pool_traffic(r["shape"]),
                                  steps=steps),
        "sequential_plain": None if ms_seq is None else {
            "value": round(lups / (ms_seq / 1e3) / 1e6, 1), "unit": "MLUPS", "ms": round(ms_seq, 2),
            "launch_shape_of_first_lattice": r["seq_launch"]},
        "speedup_vs_sequential": None if ms_seq is None else round(ms_seq / r["ms_batched"], 3),
        "bitwise_equal_to_sequential": None if r["equal"] is None else bool(r["equal"]),
    }


def bench_batch256(args):
    """256 independent lattices (sides log-uniform in [64, 1024], sampled
    stable rates, one pulse each, FP32, 500 steps): the whole job in one pool
    against the same 256 lattices run one after another with each lattice's
    default launches.  The two give bit-identical fields (checked)."""
    import lbm_inputs
    w = lbm_inputs.WORKLOADS["batch256"]
    steps = w["steps"] if args.steps == 2000 else args.steps
    shape = parse_pool_shape(args.pool_shape) if args.pool_shape else None
    r = run_batch256(steps, shape, sequential=not args.no_sequential)
    summ = batch_summary(r, steps)
    return {
        "metric": METRIC, "value": summ["value"], "unit": "MLUPS", "n_gpus": 1,
        "steps": steps, "warmup": steps, "ms_per_step": summ["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch256", "lattices": r["lattices"], "cells": r["cells"], "steps": steps,
                   "seed": r["seed"], "pool_shape": r["shape"], "stability_draws": r["draws"],
                   "stability_acceptance": round(r["lattices"] / r["draws"], 4)},
        "roofline": summ["roofline"],
        "sequential_plain": summ["sequential_plain"],
        "speedup_vs_sequential": summ["speedup_vs_sequential"],
        "bitwise_equal_to_sequential": summ["bitwise_equal_to_sequential"],
        "context": {"copy_probe": copy_probe(603979776, 10)},
    }


def serve_warmup(budget):
    """Untimed warm-up of the serving modes: the first use of each kernel,
    pool graph and allocation size in the process is not charged to the
    first measured trace."""
    import lbm_inputs
    from paper_1107_4543_amd import stability
    from paper_1107_4543_amd.serve import Server, run_plain
    warm = lbm_inputs.serving_trace(99, 1000.0, 24, accept=stability.stable)
    for policy in ("aged", "fifo"):
        srv = Server(budget, max_members=256, policy=policy, keep="digest")
        srv.run(warm)
        srv.close()
    run_plain(warm, keep="digest")


def serve_rate(seed, rate, jobs, budget, policies):
    """One Poisson trace (seed, rate in jobs/s, jobs) served under each
    admission policy and run one job at a time; every job's final raw state
    is compared between the modes through its on-device digest.  The first
    policy is the one reported as "served"."""
    import lbm_inputs
    from paper_1107_4543_amd import stability
    from paper_1107_4543_amd.serve import Server, run_plain, summarize
    trace = lbm_inputs.serving_trace(seed, rate, jobs, accept=stability.stable)
    modes, peak = {}, {}
    for policy in policies:
        srv = Server(budget, max_members=256, policy=policy, keep="digest")
        modes[policy] = srv.run(trace)
        srv.close()
        peak[policy] = (srv.peak_members, round(srv.peak_used / 1e9, 2), len(srv.rejected))
    plain = run_plain(trace, keep="digest")
    pd = {r.tag: r.digest for r in plain}
    mismatched = sorted({r.tag for rs in modes.values() for r in rs if r.digest != pd.get(r.tag)})
    first = policies[0]
    row = {"rate_jobs_per_s": rate, "jobs": len(trace), "seed": seed, "served": summarize(modes[first]),
           **{"served_" + p: summarize(modes[p]) for p in policies[1:]},
           "plain": summarize(plain),
           "equal_results": not mismatched and all(len(rs) == len(trace) for rs in modes.values()),
           "jobs_compared": sum(len(rs) for rs in modes.values()), "mismatched_jobs": mismatched,
           "rejected": peak[first][2], "peak_members": peak[first][0], "peak_budget_gb": peak[first][1]}
    return row


def bench_serve(args):
    """Poisson arrivals of simulation jobs (square side log-uniform in
    [128, 4096], steps uniform in [200, 5000], FP32 or FP16 storage 50/50,
    sampled stable rates, pulse or plane-wave initial fields), served with
    continuous batching under an HBM budget (admission: shortest job first
    with ageing, the server's default; also plain shortest job first and
    arrival order) and, on the same trace, one job at a time with each
    lattice's default launches.  Latency = arrival to result on the host.
    Every job's final raw state is compared between the modes through an
    on-device digest of its stored values."""
    out = []
    budget = int(args.budget_gb * 1e9)
    serve_warmup(budget)
    for i, rate in enumerate(float(r) for r in args.rates.split(",")):
        row = serve_rate(100 + i, rate, args.jobs, budget, ("aged", "sjf", "fifo"))
        out.append(row)
        print(json.dumps({"progress": row}), file=sys.stderr, flush=True)
    top = out[-1]["served"]
    return {"metric": METRIC, "value": top["aggregate_mlups"], "unit": "MLUPS", "n_gpus": 1,
            "steps": None, "warmup": 0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32/f16", "data": "synthetic",
            "config": {"workload": "serve", "jobs_per_rate": args.jobs, "budget_gb": args.budget_gb,
                       "rates": args.rates, "admission": "aged shortest-job-first (also sjf, fifo)",
                       "pools": "FP32/FP64 jobs (7 steps per launch) and 16-bit jobs (6 per launch), "
                                "a job alone with its own launches"},
            "serving": out}


def bench_pulses8192(args):
    """Precision study: 8192 x 8192, Lallemand-Luo rates (nu = 1e-3), 16 seeded
    Gaussian pulses, 1000 steps, for each storage type (FP64 with FP64 and
    with FP32 collide, FP32, FP16, BF16 with FP32 collide): MLUPS and roofline
    of the tuned step kernel, and the density error against the FP64 run
    (which the tests check against the oracle on sampled windows)."""
    import torch

    import lbm_inputs
    from paper_1107_4543_amd import Lattice
    w = lbm_inputs.WORKLOADS["pulses8192"]
    nx, ny = w["nx"], w["ny"]
    T = w["steps"] if args.steps == 2000 else args.steps
    ll = lbm_inputs.PRESETS["LL"]
    s = [ll["s_e"], ll["s_eps"], ll["s_q"], 1.0 / (3.0 * w["nu"] + 0.5)]
    specs = lbm_inputs.random_pulse_specs(nx, ny, w["seed"], w["count"])
    dev = "cuda:0"
    fields = lbm_inputs.pulses_field_torch(nx, ny, specs, dev)
    A = float((fields[0] - 1.0).abs().max())
    rows, rho_ref = [], None
    for storage, compute in [("f64", "f64"), ("f64", "f32"), ("f32", "f32"), ("f16", "f32"), ("bf16", "f32")]:
        lat = Lattice(nx, ny, *s, storage=storage, compute=compute, device=dev).init(*fields)
        launch, _ = lat.tune(reps=3)
        lat.init(*fields)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(T)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        rho = lat.moments()[0]
        if rho_ref is None:
            rho_ref = rho
            e_inf = e_l2 = 0.0
        else:
            d = rho - rho_ref
            e_inf = float(d.abs().max()) / A
            e_l2 = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(rho_ref - 1.0))
        spl = lat.steps_per_launch
        launches = lat.launches_for(T)
        # every launch reads and writes all nine planes once, whether it
        # advances one step or several
        bpl = 18 * STORE_BYTES[storage] * launches / T
        gbps = 18 * STORE_BYTES[storage] * nx * ny * launches / (ms / 1e3) / 1e9
        mlups_r = nx * ny * T / (ms / 1e3) / 1e6
        alu_tops = alg_ops_per_lu(storage, compute) * mlups_r * 1e6 / 1e12
        rows.append({"storage": storage, "compute": compute, "mlups": round(mlups_r, 1),
                     "alg_ops_TOPs": round(alu_tops, 2), "alu_frac": round(alu_tops * 1e12 / ALU_PEAK[compute], 4),
                     "bytes_per_lu": round(bpl, 3), "achieved_GBps": round(gbps, 1),
                     "frac": round(gbps / HBM_PEAK_GBPS, 4), "launch": launch, "steps_per_launch": spl,
                     "scale_exp": lat.scale_exp,
                     "linf_err_over_A": e_inf, "l2_rel_err": e_l2})
        print(json.dumps({"progress": rows[-1]}), file=sys.stderr, flush=True)
        del lat, rho
    best = max(rows, key=lambda r: r["mlups"])
    return {"metric": METRIC, "value": best["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": T, "warmup": 0,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": best["storage"],
            "data": "synthetic",
            "config": {"workload": "pulses8192", "nx": nx, "ny": ny, "pulses": w["count"], "seed": w["seed"],
                       "relaxation": "Lallemand-Luo, nu = 1e-3", "amplitude_max": A},
            "precision": rows}


def parse_launch(text):
    keys = ["variant", "block_x", "block_y", "rows", "xcd_remap", "flags"]
    vals = [int(v) for v in text.split(",")]
    if len(vals) != len(keys):
        raise SystemExit("--launch takes variant,block_x,block_y,rows,xcd_remap,flags")
    return dict(zip(keys, vals))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16", "bf16"])
    ap.add_argument("--workload", default="waves4096", choices=["waves4096", "batch256", "serve", "pulses8192"],
                    help="waves4096: one 4096^2 lattice (default); batch256: 256 lattices, pool vs "
                         "sequential; serve: Poisson job traces, continuous batching vs plain FIFO")
    ap.add_argument("--rates", default="10,30,100,300,1000", help="serve: arrival rates (jobs/s)")
    ap.add_argument("--jobs", type=int, default=200, help="serve: jobs per rate")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve: HBM budget for admitted jobs")
    ap.add_argument("--no-tune", action="store_true", help="use the library's default launch shape (several steps per launch from 2^19 cells)")
    ap.add_argument("--tune", action="store_true", help="search the launch shape with lbm_tune before timing")
    ap.add_argument("--launch", default=None,
                    help="launch shape variant,block_x,block_y,rows,xcd_remap,flags (default: the recorded "
                         "tuned shape for the storage type)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch256: skip the one-lattice-at-a-time comparison (for counter profiling)")
    ap.add_argument("--pool-shape", default=None,
                    help="batch256: pool shape tile_cells,block,grid,graph_steps,steps_per_launch,seg_rows,waves,"
                         "flags (no tuning)")
    ap.add_argument("--probe", choices=["copy"], default=None,
                    help="run only the device-to-device copy probe")
    ap.add_argument("--probe-bytes", type=int, default=1 << 30)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work (0 = skip)")
    ap.add_argument("--cpu-budget-1t", type=float, default=5.0,
                    help="seconds of one-thread oracle work (0 = skip)")
    ap.add_argument("--batched-steps", type=int, default=500,
                    help="default workload: steps of the batched 256-lattice run reported beside it (0 = skip)")
    ap.add_argument("--served-jobs", type=int, default=100,
                    help="default workload: jobs of the served-vs-plain trace reported beside it (0 = skip)")
    ap.add_argument("--served-rate", type=float, default=1000.0,
                    help="default workload: arrival rate (jobs/s) of that trace")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the lattice path runs on one GPU "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()

    if args.probe == "copy":
        print(json.dumps({"probe": "copy", **copy_probe(args.probe_bytes, args.steps)}), flush=True)
        return
    if args.workload == "batch256":
        print(json.dumps(bench_batch256(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "pulses8192":
        print(json.dumps(bench_pulses8192(args)), flush=True)
        return

    lat, cfg, rates, fields1, w = build_waves4096(args.storage)
    if args.tune:
        lat.tune(reps=5)
    elif not args.no_tune:
        lat.set_launch(**parse_launch(args.launch or DEFAULT_LAUNCH[args.storage]))
    cfg["launch"] = lat.launch

    stream = lat.stream
    lat.step(args.warmup)
    spl = lat.steps_per_launch
    torch.cuda.synchronize()
    # The timed region is args.steps steps on the lattice's stream.  With a
    # several-steps shape it is issued one launch of spl steps at a time, a
    # HIP event after each, so the dominant kernel's own launches are timed
    # apart from the one shorter launch that takes the steps left over.
    full, rest = (args.steps // spl, args.steps % spl) if spl > 1 else (0, args.steps)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(full + 2)]
    ev[0].record(stream)
    for i in range(full):
        lat.step(spl)
        ev[i + 1].record(stream)
    if rest:
        lat.step(rest)
    ev[full + 1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[full + 1])
    st, diag = lat.diagnostics()
    assert st == 0, "non-finite state after the timed steps"

    cells = lat.nx * lat.ny
    mlups = cells * args.steps / (ms / 1e3) / 1e6
    launches = lat.launches_for(args.steps)             # T-step launches and the left-over one(s)
    alg_bytes = 2 * 9 * STORE_BYTES[args.storage] * cells
    traffic = read_traffic("waves4096", args.storage, lat.launch)

    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic", "config": cfg,
    }
    # one pass per step would move 2 * 9 * sizeof(storage) bytes per update:
    # the bytes a one-pass kernel needs for this many updates per second
    one_pass = alg_bytes * args.steps / (ms * 1e-3) / 1e9
    one_pass_equiv = {"achieved": round(one_pass, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                      "frac": round(one_pass / HBM_PEAK_GBPS, 4),
                      "bytes_per_update": 2 * 9 * STORE_BYTES[args.storage]}
    if spl == 1:
        # one step per launch: every update reads and writes all nine planes
        us = 1e3 * ms / launches
        achieved = alg_bytes / (us * 1e-6) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                           "algorithmic_bytes_per_launch": alg_bytes,
                           "kernel": "k_step (fused collide + pull stream)", "steps_per_launch": 1,
                           "launches": launches, "avg_launch_us": round(us, 3)}
    else:
        # several steps per launch move a T-th of the bytes per update; the
        # bound is the vector ALU: the collision's algorithmic operations of
        # the spl steps one launch of the dominant kernel advances, over that
        # kernel's average launch duration (its own launches' events),
        # against the non-packed issue peak of the compute type
        compute = lat.compute
        peak = ALU_PEAK[compute] / 1e12
        # (fewer steps than one launch: the region's single shorter launch)
        us = 1e3 * ev[0].elapsed_time(ev[full]) / full if full else 1e3 * ms / launches
        ops_lu = alg_ops_per_lu(args.storage, compute)
        ops = ops_lu * cells * spl
        tops = ops / (us * 1e-6) / 1e12
        # the same over the whole timed region, from the steps actually run
        tops_all = ops_lu * cells * args.steps / (ms * 1e-3) / 1e12
        achieved_b = alg_bytes / (us * 1e-6) / 1e9
        hbm = {"bound": "hbm", "achieved": round(achieved_b, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
               "frac": round(achieved_b / HBM_PEAK_GBPS, 4), "traffic": traffic,
               "algorithmic_bytes_per_launch": alg_bytes,
               "reading": "bytes one launch of the dominant kernel moves (it reads and writes every "
                          "population once for spl steps) over its average launch duration"}
        out["roofline"] = {"bound": "alu", "achieved": round(tops, 2), "peak": round(peak, 2),
                           "unit": "T %s ops/s" % compute.upper(), "frac": round(tops / peak, 4),
                           "traffic": traffic, "algorithmic_ops_per_launch": ops,
                           "ops_per_update": ops_lu,
                           "kernel": "k_step_multi (%d steps per pass)" % spl, "steps_per_launch": spl,
                           "launches_timed": full, "avg_launch_us": round(us, 3),
                           "timed_region": {"steps": args.steps, "launches": launches, "ms": round(ms, 4),
                                            "achieved": round(tops_all, 2), "frac": round(tops_all / peak, 4),
                                            "leftover_launch_steps": rest},
                           "hbm": hbm, "one_pass_equiv": one_pass_equiv}
        kv = read_profile("waves4096", args.storage, lat.launch)
        if kv and "valu_lane_instructions_per_update" in kv:
            # what the compiled loop issues per useful update (halo lanes,
            # prologue rows and register moves included), see the profile
            per_lu = float(kv["valu_lane_instructions_per_update"])
            rate = cells * spl / (us * 1e-6)
            out["roofline"]["valu_issue"] = {"lane_instructions_per_update": per_lu,
                                             "achieved": round(per_lu * rate / 1e12, 2),
                                             "peak": round(VALU_PEAK / 1e12, 2), "unit": "T lane-instr/s",
                                             "frac": round(per_lu * rate / VALU_PEAK, 4)}
    if spl == 1:
        out["roofline"]["one_pass_equiv"] = one_pass_equiv
    out["context"] = {"copy_probe": copy_probe(alg_bytes // 2, 10), "device": torch.cuda.get_device_name(0)}
    del lat
    if args.batched_steps > 0:
        # the batched workload (256 lattices) with the recorded pool shape
        import lbm_inputs
        shape = parse_pool_shape(args.pool_shape or DEFAULT_POOL_SHAPE)
        r = run_batch256(args.batched_steps, shape, sequential=True)
        out["batched"] = dict({"workload": "batch256", "lattices": r["lattices"], "cells": r["cells"],
                               "seed": r["seed"], "pool_shape": r["shape"],
                               "job_steps": lbm_inputs.WORKLOADS["batch256"]["steps"]},
                              **batch_summary(r, args.batched_steps))
    if args.served_jobs > 0:
        # one Poisson trace served with continuous batching (aged shortest job
        # first, the server's default) and one job at a time, same jobs
        budget = int(args.budget_gb * 1e9)
        serve_warmup(budget)
        row = serve_rate(100, args.served_rate, args.served_jobs, budget, ("aged",))
        out["serving"] = dict({"workload": "serve", "budget_gb": args.budget_gb,
                               "admission": "aged shortest-job-first",
                               "pools": "FP32/FP64 jobs (7 steps per launch) and 16-bit jobs (6 per launch), "
                                        "a job alone with its own launches"}, **row)
    if args.cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline(rates, fields1, cfg["nx"], cfg["ny"], w["u0x"], args.cpu_budget,
                                           args.cpu_budget_1t)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
