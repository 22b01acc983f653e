"""Throughput benchmark: parallel-tempering Metropolis on one MI355X.

Workload (default): 2D Ising 1024x1024, J = 1, h = 0, R = 64 replicas with beta
linear in [0.30, 0.55], spins drawn from seed 2; E_int and M reduced and
recorded after every sweep; one replica-exchange step every 10 sweeps.
A step is one interval of that schedule (10 checkerboard sweeps of all 64
replicas + their records + one exchange step, i.e. 6.7e8 flip attempts); the
full run of the workload is 1000 steps (10^4 sweeps), timed as one pt_run call
of the whole schedule (the library splits it into launches).

Prints one JSON line: flip attempts/s of the whole job, the roofline of the
sweep kernel (integer-VALU bound; average launch duration measured live with
HIP events on the library's stream), and the CPU oracle timed on a bounded
sample of the same workload on one host core.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 compute units x 4 SIMD x 16 lanes at 2.4 GHz = 39.3e12 VALU lane
# slots per second for 32-bit integer operations (one wave64 instruction per SIMD
# every four clocks).  On gfx950 the 32x32->64 multiply-add (v_mad_u64_u32) and
# the three-input XOR (v_bitop3_b32) are full-rate instructions (their measured
# issue rates are what `--form probe` reports).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# LDS: 128 bytes per clock per compute unit.
LDS_PEAK_TBPS = 256 * 128 * 2.4e9 / 1e12
HBM_PEAK_TBPS = 8.0
# Least VALU work of one flip attempt under the method's draw contract, the
# roofline's algorithmic figure: a quarter of a Philox4x32-10 block -- per round
# two 32x32->64 products and two three-input XORs, one instruction each; the
# counter words 1-3 (sweep, slot, colour) and the key are the same for every
# lane, so the first round's second product, the second round's first product
# and the XORs they feed are scalar work, leaving 18 products + 19 XORs = 37
# vector instructions per block of four draws -- and one compare of each draw
# with its threshold.  No kernel that consumes one Philox word per attempt
# issues fewer, whatever its stencil, tallies and layout cost on top (the
# kernels issue ~17.5 per attempt in all; the counters give the exact figure).
PHILOX_VALU_PER_BLOCK = 37
SLOTS_PER_ATTEMPT = PHILOX_VALU_PER_BLOCK / 4 + 1
# LDS bytes one attempt moves in the main kernels (loads and stores per item,
# counted from the code).  2D span of 8 nibble dwords (32 attempts): the row,
# the rows above and below (32 B each), one edge dword, 32 table reads, the
# store (32 B): 260 B with 4-byte thresholds (the 2D split kernel), 388 B with
# the 8-byte compare entries (tiled kernels).  Phased span of 4 dwords (16
# attempts): the row (16 B), 5 dwords of each neighbour row, an edge dword, 16
# 8-byte entries, the store: 204 B.  3D span of 4 dwords (16 attempts): spins
# and x bonds (16 B each), edge spin and bond, rows y -+ 1 and their y bonds,
# planes z -+ 1 and their z bonds (8 x 16 B), 16 8-byte entries, the store:
# 312 B.
LDS_BYTES_PER_ATTEMPT = {"k_persist_split/2": 260 / 32, "k_tiled_n/2": 388 / 32,
                         "k_phased/2": 204 / 16, "k_persist_split/3": 312 / 16,
                         "k_tiled/3": 312 / 16, "k_persist/2": 388 / 32, "k_persist/3": 312 / 16}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ising2d_L1024_R64")
    ap.add_argument("--plan", choices=["auto", "fused", "tiled", "persistent", "lanes", "wave"],
                    default="auto", help="launch decomposition (every plan gives identical results)")
    ap.add_argument("--tile-planes", type=int, default=0)
    ap.add_argument("--sweeps-per-launch", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--exchange-every", type=int, default=-1,
                    help="plain form: override the workload's exchange interval in sweeps "
                         "(0: no exchange steps; -1: the workload's own)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=4)
    ap.add_argument("--form", choices=["plain", "batched", "served", "physics", "probe"], default="plain",
                    help="plain: one PT instance (the default workload); batched: 2048 "
                         "independent instances advanced together, against the per-instance path; "
                         "served: a Poisson stream of jobs through the request loop; physics: "
                         "|M|/N and E/N against T and sweeps-to-equilibrium against L; probe: "
                         "issue rates of the VALU instructions the sweep kernels are built from")
    ap.add_argument("--batch-instances", type=int, default=2048)
    ap.add_argument("--batch-sweeps", type=int, default=2000)
    ap.add_argument("--jobs", type=int, default=400, help="served form: jobs in the stream")
    ap.add_argument("--job-range", default="",
                    help="served form: serve only jobs a..b-1 of the stream ('a:b'), arriving at their "
                         "times in the whole stream shifted so that job a arrives first")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="served form: arrival rate in jobs/s (0: rho x measured capacity / mean job)")
    ap.add_argument("--plain-sample", type=int, default=100,
                    help="served form: jobs of the stream also served one at a time by the plain "
                         "path, end to end at their arrival times (0: none)")
    ap.add_argument("--latencies-out", default="",
                    help="served form: write every job's arrival, finish and size to this JSON file")
    ap.add_argument("--rho", type=float, default=0.8, help="served form: offered load / capacity")
    ap.add_argument("--arena-gib", type=float, default=8.0, help="served form: job arena (GiB)")
    ap.add_argument("--tiled-lanes", type=int, default=1, help="served form: streams for large lattices")
    ap.add_argument("--class-sites", default="4096,65536",
                    help="served form: ascending sites-per-replica bounds of the batched lanes' size "
                         "classes, comma-separated (empty: one batched lane)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 64 MiB device-to-device copy (a kernel of known "
                         "traffic, to scale HBM counters)")
    return ap.parse_args()


KERNEL_SOURCES = ("paper_2512_03825_amd/csrc/pt_kernels.hip", "paper_2512_03825_amd/csrc/pt_internal.h")


def kernel_source_hash():
    """sha256 over the device-kernel sources (ties an HBM counter reading to the code it measured)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_fields(kernel, workload, plan, per_launch, suffix=""):
    """The `- key: value` lines of profiles/<kernel>_<workload><suffix>.md when
    that summary was taken on these kernel sources, this plan and this launch
    length; None otherwise (or when there is no such summary)."""
    path = os.path.join(ROOT, "profiles", "%s_%s%s.md" % (kernel, workload, suffix))
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                fields[k] = v.strip("` ")
    want = {"kernel_source_sha256": kernel_source_hash(),
            "plan": "mode=%d tile_planes=%d sweeps_per_launch=%d block_threads=%d" % (
                plan["mode"], plan["tile_planes"], plan["sweeps_per_launch"], plan["block_threads"]),
            "sweeps_per_launch_measured": str(per_launch)}
    if any(fields.get(k) != v for k, v in want.items()):
        return None
    return fields


def measured_traffic(kernel, workload, plan, per_launch):
    """HBM bytes per launch of `kernel` from the FETCH_SIZE / WRITE_SIZE passes
    summarised under profiles/ (each counter scaled by what it reads for a plain
    copy of known size), or None."""
    f = profile_fields(kernel, workload, plan, per_launch)
    return int(f["traffic_bytes_per_launch"]) if f and "traffic_bytes_per_launch" in f else None


def measured_valu_insts(kernel, workload, plan, per_launch):
    """VALU wave-instructions per launch (SQ_INSTS_VALU) from the SQ counter
    summary under profiles/, or None."""
    f = profile_fields(kernel, workload, plan, per_launch, "_sq")
    return float(f["valu_insts_per_launch"]) if f and "valu_insts_per_launch" in f else None


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def pinned(fn):
    """Run fn() with this process pinned to one host core (the oracle is
    single-threaded); returns (result, core)."""
    try:
        before = os.sched_getaffinity(0)
    except (AttributeError, OSError):
        return fn(), None
    core = min(before)
    os.sched_setaffinity(0, {core})
    try:
        return fn(), core
    finally:
        os.sched_setaffinity(0, before)


def cpu_baseline(w, sweeps, every):
    """The CPU oracle, as it stands, on a bounded prefix of the same workload,
    on one host core."""
    import oracle
    o = oracle.Oracle(w.model, w.L, w.R, w.beta, seed=w.seed, coupling_seed=w.coupling_seed)

    def go():
        t0 = time.perf_counter()
        o.run(sweeps, every)
        return time.perf_counter() - t0

    dt, core = pinned(go)
    attempts = sweeps * w.attempts_per_sweep
    return {"value": attempts / dt, "unit": "flip attempts/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu(), "host_cpus": os.cpu_count(), "pinned_core": core,
            "sample": "%s: first %d sweeps after initialisation (%.3g flip attempts, %.1f s, "
                      "single thread pinned to one core)" % (w.name, sweeps, attempts, dt)}


def bench_batched(args):
    """Batched form: every instance advanced by the same schedule in one batch,
    timed against running the same instances one after another."""
    import torch

    from paper_2512_03825_amd import pt
    from paper_2512_03825_amd.workloads import batched2048

    ws = batched2048(n=args.batch_instances)
    every, sweeps = ws[0].exchange_every, args.batch_sweeps
    cfgs = [pt.Config(w.model, w.L, w.R, w.beta, h=w.h, seed=w.seed, stream_id=w.stream_id)
            for w in ws]
    torch.cuda.set_device(0)
    batch = pt.Batch(cfgs, device="cuda:0")
    # warm-up: the tuning cycles of the first run pick each group's decomposition
    batch.run(10 * every, every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.run(sweeps, every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    attempts = sweeps * sum(w.attempts_per_sweep for w in ws)
    plans = batch.group_plans()
    batch.close()
    del batch
    # the plain per-instance path on the same instances (a prefix of the schedule each)
    per_sweeps = 4 * every
    sims = [pt.Simulation(c, device="cuda:0") for c in cfgs]
    for s in sims:
        s.run(every, every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.run(per_sweeps, every)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t0
    single = per_sweeps * sum(w.attempts_per_sweep for w in ws) / dt1
    for s in sims:
        s.close()
    out = {"metric": "spin-flip attempts/s", "value": attempts / dt, "unit": "flip attempts/s",
           "n_gpus": 1, "steps": sweeps // every, "warmup": 10, "ms_per_step": dt / (sweeps / every) * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
           "data": "synthetic",
           "config": {"workload": "batched%d" % len(ws), "instances": len(ws), "sweeps": sweeps,
                      "exchange_every": every, "L": sorted({w.L for w in ws}),
                      "R": sorted({w.R for w in ws}), "h": [-0.1, 0.1], "group_plans": plans,
                      # with h != 0 the exchange is the paper's logistic test on the
                      # h = 0 exponent times a Metropolis test on the field term
                      # (detailed balance for the full exponent; the paper's rule at h = 0)
                      "swap_rule": "h != 0: logistic(beta-difference x bond-energy difference)"
                                   " x Metropolis(field term), not one logistic test",
                      "parallelism": "single GPU"},
           "per_instance_path": {"value": single, "unit": "flip attempts/s",
                                 "sample": "same %d instances one after another, %d sweeps each"
                                           % (len(ws), per_sweeps)},
           "speedup_vs_per_instance": (attempts / dt) / single,
           "roofline": batched_roofline(attempts / dt)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_instances(ws[:16], 20)
    print(json.dumps(out), flush=True)


def batched_roofline(rate, slots=SLOTS_PER_ATTEMPT):
    """Whole-cycle VALU roofline of a batched or served run: attempts/s times
    the algorithmic lane slots per attempt, against the VALU peak (exchange
    and counter launches are inside the time)."""
    achieved = rate * slots / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "Tops/s (int32 VALU lane slots)", "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "traffic": None, "kernel": "k_batch_sweep (whole cycle)",
            "slots_per_attempt": round(slots, 3)}


def cpu_baseline_instances(ws, sweeps):
    """The CPU oracle on a bounded sample: the first instances of the list, a
    prefix of each one's schedule, one after another on one core."""
    import oracle

    def go():
        t = 0.0
        attempts = 0
        for w in ws:
            o = oracle.Oracle(w.model, w.L, w.R, w.beta, J=w.J, h=w.h, seed=w.seed,
                              stream_id=w.stream_id, coupling_seed=w.coupling_seed)
            n = min(sweeps, w.sweeps)
            t0 = time.perf_counter()
            o.run(n, w.exchange_every)
            t += time.perf_counter() - t0
            attempts += n * w.attempts_per_sweep
        return t, attempts

    (t, attempts), core = pinned(go)
    return {"value": attempts / t, "unit": "flip attempts/s", "cores": 1, "kind": "oracle",
            "host_cpu": host_cpu(), "host_cpus": os.cpu_count(), "pinned_core": core,
            "sample": "first %d instances, %d sweeps each (%.3g flip attempts, %.1f s, single "
                      "thread pinned to one core)" % (len(ws), sweeps, attempts, t)}


def _serve(pt, srv, cfgs, ws, arrivals, t_label):
    """Submit job i at arrivals[i] seconds (server clock) and run the request
    loop until every job has finished; returns the finished-job records."""
    n = len(cfgs)
    t0 = srv.clock()
    nxt, out, last_note = 0, [], time.time()
    while len(out) < n:
        now = srv.clock() - t0
        while nxt < n and arrivals[nxt] <= now:
            srv.submit(cfgs[nxt], ws[nxt].sweeps, ws[nxt].exchange_every, arrival=t0 + arrivals[nxt])
            nxt += 1
        wait = 2000 if nxt >= n else int(max(0.0, min(2e-3, arrivals[nxt] - now)) * 1e6)
        srv.step(wait_us=wait)
        for f in srv.done():
            f["arrival"] -= t0
            f["finished"] -= t0
            f["admitted"] -= t0
            out.append(f)
            srv.release(f["job_id"])
        if time.time() - last_note > 10:
            st = srv.stats()
            print("[%s] t=%.1fs submitted %d finished %d resident %d pending %d" % (
                t_label, now, nxt, len(out), st["resident"], st["pending"]), file=sys.stderr, flush=True)
            last_note = time.time()
    return out


def _plain_fifo(pt, cfgs, ws, arrivals):
    """The plain per-instance path on the same arrivals, one job at a time in
    arrival order (first come, first served), each job created and run with
    pt_run at its full length when the previous one has finished; returns the
    latencies (finish - arrival) and the summed service time."""
    import torch
    lat, busy = [], 0.0
    t0 = time.perf_counter()
    last_note = time.time()
    for i, (w, c) in enumerate(zip(ws, cfgs)):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        t1 = time.perf_counter()
        sim = pt.Simulation(c, device="cuda:0")
        sim.run(w.sweeps, w.exchange_every)
        torch.cuda.synchronize()
        sim.close()
        del sim
        t2 = time.perf_counter()
        busy += t2 - t1
        lat.append(t2 - t0 - arrivals[i])
        if time.time() - last_note > 10:
            print("[plain per-instance] %d of %d jobs, t=%.1fs" % (i + 1, len(ws), t2 - t0),
                  file=sys.stderr, flush=True)
            last_note = time.time()
    return lat, busy


def bench_served(args):
    """Served form: a Poisson stream of PT jobs through the request loop at
    offered load rho of the server's measured capacity; p50/p99 latency and
    aggregate flips/s, beside the plain per-instance path serving a sample of
    the same stream one job at a time (first come, first served), end to end."""
    import numpy as np
    import torch

    from paper_2512_03825_amd import pt
    from paper_2512_03825_amd.workloads import poisson_arrivals, served_jobs

    torch.cuda.set_device(0)
    all_ws = served_jobs(n=args.jobs)
    a, b = 0, len(all_ws)
    if args.job_range:
        a, b = (int(x) for x in args.job_range.split(":"))
        if not 0 <= a < b <= len(all_ws):
            raise SystemExit("--job-range %s outside the %d-job stream" % (args.job_range, len(all_ws)))

    def config(w):
        return pt.Config(w.model, w.L, w.R, w.beta, J=w.J, h=w.h, seed=w.seed, stream_id=w.stream_id,
                         coupling_seed=w.coupling_seed, record_every=w.record_every,
                         max_records=w.sweeps // w.record_every)

    att_all = np.array([w.attempts_per_sweep * w.sweeps for w in all_ws], dtype=np.float64)
    opts = dict(max_jobs=4096, max_walkers=1 << 20, tiled_lanes=args.tiled_lanes, depth=2,
                cycle_sweeps=10, tiled_sweeps=5, class_sites=[int(x) for x in args.class_sites.split(",") if x])
    srv = pt.Server(int(args.arena_gib * (1 << 30)), device="cuda:0", **opts)
    # capacity: the first 200 jobs of the stream cut to 2000 sweeps, all submitted at once
    import copy
    cut = []
    for w in all_ws[:200]:
        w2 = copy.copy(w)
        w2.sweeps = min(w.sweeps, 2000)
        cut.append(w2)
    t = time.perf_counter()
    _serve(pt, srv, [config(w) for w in cut], cut, np.zeros(len(cut)), "capacity")
    cap_dt = time.perf_counter() - t
    C = sum(w.attempts_per_sweep * w.sweeps for w in cut) / cap_dt
    lam = args.rate if args.rate > 0 else args.rho * C / att_all.mean()
    arrivals_all = poisson_arrivals(lam, len(all_ws))
    ws = all_ws[a:b]
    cfgs = [config(w) for w in ws]
    att = att_all[a:b]
    arrivals = arrivals_all[a:b] - arrivals_all[a]
    t = time.perf_counter()
    fin = _serve(pt, srv, cfgs, ws, arrivals, "served rho=%.2f" % args.rho)
    dt = time.perf_counter() - t
    srv.close()
    fin.sort(key=lambda f: f["job_id"])
    lat = np.array([f["finished"] - f["arrival"] for f in fin])
    span = max(f["finished"] for f in fin) - min(f["arrival"] for f in fin)
    value = att.sum() / span
    if args.latencies_out:
        with open(args.latencies_out, "w") as fh:
            json.dump({"jobs": [a, b], "rate": lam, "arrival": [f["arrival"] for f in fin],
                       "finished": [f["finished"] for f in fin], "attempts": att.tolist(),
                       "lane": [f["lane"] for f in fin]}, fh)

    # the plain per-instance path, end to end on a sample: the first jobs of
    # the segment at the same arrival times, one at a time
    m = min(args.plain_sample, len(ws))
    plain_lat, busy = _plain_fifo(pt, cfgs[:m], ws[:m], arrivals[:m]) if m else ([], 0.0)
    plain_capacity = float(att[:m].sum() / busy) if m else None
    out = {"metric": "served-job latency p50/p99 + flip attempts/s", "value": value,
           "unit": "flip attempts/s", "n_gpus": 1, "steps": len(ws), "warmup": 0,
           "ms_per_step": dt / len(ws) * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "served%d" % len(all_ws), "jobs": [a, b], "rho": args.rho,
                      "arrival_rate_per_s": lam, "mean_attempts_per_job": float(att_all.mean()),
                      "server": opts, "arena_bytes": int(args.arena_gib * (1 << 30)),
                      "parallelism": "single GPU"},
           "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                         "max": float(lat.max())},
           "capacity": {"served": C, "plain_per_instance": plain_capacity,
                        "sample": "served: first %d jobs cut to 2000 sweeps, all at t=0 (%.1f s); "
                                  "plain: the segment's first %d jobs run end to end one at a time "
                                  "(%.1f s of service)" % (len(cut), cap_dt, m, busy)},
           "plain_fifo_latency_s": ({"jobs": m, "p50": float(np.percentile(plain_lat, 50)),
                                     "p99": float(np.percentile(plain_lat, 99)),
                                     "max": float(max(plain_lat))} if m else None),
           "served_latency_same_jobs_s": ({"p50": float(np.percentile(lat[:m], 50)),
                                           "p99": float(np.percentile(lat[:m], 99))} if m else None),
           "speedup_vs_per_instance": C / plain_capacity if m else None,
           "roofline": batched_roofline(C)}
    out["roofline"]["kernel"] = "served capacity (batched and tiled lanes)"
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_instances(ws[:8], 20)
    print(json.dumps(out), flush=True)


def onsager_energy(beta):
    """Energy per site of the infinite 2D Ising model (J = 1, h = 0), Onsager 1944."""
    import math

    from scipy.special import ellipk
    t = math.tanh(2 * beta)
    k = 2 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2
    return -(1 / t) * (1 + (2 / math.pi) * (2 * t * t - 1) * ellipk(k * k))


def yang_magnetisation(beta):
    """Spontaneous magnetisation per site (Yang 1952); 0 above the critical temperature."""
    import math
    x = math.sinh(2 * beta) ** -4
    return (1 - x) ** 0.125 if x < 1 else 0.0


def _blocked(x, blocks=20):
    """Mean and its standard error from `blocks` contiguous block means."""
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    n = len(x) // blocks * blocks
    b = x[len(x) - n:].reshape(blocks, -1).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / np.sqrt(blocks))


def bench_physics(args):
    """The paper's validation figures, computed with the GPU path: |M|/N and E/N
    against T across [1, 4] beside Onsager and Yang (Fig. 3a), and the sweeps a
    random start needs to reach equilibrium at T = 2 against L (Fig. 3b)."""
    import numpy as np
    import torch

    from paper_2512_03825_amd import pt
    torch.cuda.set_device(0)
    t_start = time.perf_counter()
    # Fig. 3a analogue: L = 64, 32 temperatures linear in [1, 4], PT every 10 sweeps
    L, R, sweeps, rec = 64, 32, 100_000, 10
    T = np.array([1.0 + 3.0 * k / (R - 1) for k in range(R)])
    beta = 1.0 / T
    cfg = pt.Config(pt.PT_ISING2D, L, R, beta, seed=7, record_every=rec, max_records=sweeps // rec)
    sim = pt.Simulation(cfg, device="cuda:0")
    sim.run(sweeps, 10)
    obs = sim.observables()
    sim.close()
    N = L * L
    keep = obs["n_records"] // 2  # second half of the run
    fig_a = []
    for k in range(R):
        e, de = _blocked(obs["E_series"][keep:, k] / N)  # E_int = -sum over bonds of s s (J = 1)
        m, dm = _blocked(np.abs(obs["M_series"][keep:, k]) / N)
        fig_a.append({"T": round(float(T[k]), 4), "E_per_site": e, "E_err": de,
                      "onsager": onsager_energy(beta[k]), "absM_per_site": m, "M_err": dm,
                      "yang": yang_magnetisation(beta[k])})
    # Fig. 3b analogue: T = 2.0 slot of an 8-slot ladder over T in [2.0, 2.7],
    # random start; first sweep after which the mean E/N over the next 200
    # sweeps is within 0.5% of Onsager's value; 4 seeds per L
    target = onsager_energy(0.5)
    fig_b = []
    for L in (16, 32, 64, 128, 256):
        R, cap = 8, 200_000
        Tl = np.array([2.0 + 0.7 * k / (R - 1) for k in range(R)])
        found = []
        for seed in range(4):
            cfg = pt.Config(pt.PT_ISING2D, L, R, 1.0 / Tl, seed=100 + seed, record_every=1,
                            max_records=cap)
            sim = pt.Simulation(cfg, device="cuda:0")
            s_eq, done = None, 0
            while done < cap and s_eq is None:
                n = min(cap - done, max(2000, done))
                sim.run(n, 10)
                done += n
                e = sim.observables()["E_series"][:, 0].astype(np.float64) / (L * L)
                if len(e) >= 200:
                    w = np.convolve(e, np.ones(200) / 200, mode="valid")
                    hit = np.nonzero(np.abs(w - target) < 0.005 * abs(target))[0]
                    if len(hit):
                        s_eq = int(hit[0])
            sim.close()
            found.append(s_eq)
        ok = [f for f in found if f is not None]
        fig_b.append({"L": L, "sweeps_to_equilibrium": found,
                      "median": float(np.median(ok)) if ok else None,
                      "not_reached": len(found) - len(ok)})
    out = {"metric": "physics checks (Fig. 3a/3b analogues)", "value": None, "unit": None,
           "n_gpus": 1, "data": "synthetic", "seconds": time.perf_counter() - t_start,
           "config": {"workload": "physics", "fig3a": {"L": 64, "R": 32, "T": [1.0, 4.0],
                                                       "sweeps": 100_000, "exchange_every": 10,
                                                       "record_every": 10, "seed": 7},
                      "fig3b": {"T": 2.0, "ladder": [2.0, 2.7], "R": 8, "exchange_every": 10,
                                "criterion": "mean E/N over the next 200 sweeps within 0.5% of "
                                             "Onsager", "cap_sweeps": 200_000}},
           "fig3a": fig_a, "fig3b": fig_b}
    print(json.dumps(out), flush=True)


def bench_probe(args):
    """Issue rates of the VALU instructions the sweep kernels are built from
    (dependency-free loops over the whole chip, libptprobe.so), against the
    peak derived from the unit counts and the 2.4 GHz clock."""
    import ctypes as C

    import torch
    lib = C.CDLL(os.path.join(ROOT, "paper_2512_03825_amd", "libptprobe.so"))
    lib.ptprobe_run.restype = C.c_int
    lib.ptprobe_run.argtypes = [C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p, C.c_size_t,
                                C.c_void_p, C.POINTER(C.c_float)]
    torch.cuda.set_device(0)
    blocks, threads = 2048, 256           # 8 waves per SIMD
    out = torch.empty(blocks * threads, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    # kind, what, VALU instructions per thread and iteration, iterations
    kinds = [(0, "v_mad_u64_u32 + v_bitop3_b32 (Philox round pair)", 16, 200_000),
             (1, "v_bitop3_b32", 8, 400_000),
             (2, "v_add_u32", 8, 400_000),
             (3, "Philox4x32-10 blocks, one compare per word", None, 30_000)]
    res = []
    for kind, what, per_iter, iters in kinds:
        ms = C.c_float()
        rc = lib.ptprobe_run(kind, blocks, threads, max(1, iters // 10), C.c_void_p(out.data_ptr()),
                             out.numel(), C.c_void_p(stream), C.byref(ms))
        if rc != 0:
            raise RuntimeError("ptprobe_run(%d) returned hipError %d" % (kind, rc))
        times = []
        for _ in range(3):
            rc = lib.ptprobe_run(kind, blocks, threads, iters, C.c_void_p(out.data_ptr()), out.numel(),
                                 C.c_void_p(stream), C.byref(ms))
            if rc != 0:
                raise RuntimeError("ptprobe_run(%d) returned hipError %d" % (kind, rc))
            times.append(ms.value * 1e-3)
        t = min(times)
        r = {"kind": kind, "what": what, "seconds": t, "threads": blocks * threads, "iters": iters}
        if per_iter:
            rate = blocks * threads * per_iter * iters / t / 1e12
            r.update({"lane_ops_per_s_1e12": round(rate, 3), "frac_of_peak": round(rate / VALU_PEAK_TOPS, 4)})
        else:
            words = blocks * threads * 2 * 4 * iters / t
            r.update({"philox_words_per_s": words,
                      "frac_of_peak_at_lower_bound": round(words * SLOTS_PER_ATTEMPT / 1e12 / VALU_PEAK_TOPS, 4)})
        res.append(r)
        print("[probe] %s: %.3f ms" % (what, t * 1e3), file=sys.stderr, flush=True)
    print(json.dumps({"metric": "VALU issue-rate probe", "peak_lane_ops_per_s_1e12": round(VALU_PEAK_TOPS, 3),
                      "slots_per_attempt_lower_bound": SLOTS_PER_ATTEMPT, "results": res}), flush=True)


def main():
    args = parse()
    if args.form == "probe" and args.gpus == 1:
        return bench_probe(args)
    if args.form == "physics" and args.gpus == 1:
        return bench_physics(args)
    if args.form == "batched" and args.gpus == 1:
        return bench_batched(args)
    if args.form == "served" and args.gpus == 1:
        return bench_served(args)
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported (the path would "
              "shard by temperature slots: each GPU a block of slots, the energies all-gathered "
              "at every exchange step)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2512_03825_amd import pt
    from paper_2512_03825_amd.workloads import WORKLOADS

    w = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    every = w.exchange_every if args.exchange_every < 0 else args.exchange_every
    # a step is 10 sweeps of the workload's schedule (a whole number of
    # exchange intervals), so one step is one launch for the fused and
    # persistent plans and a few launches for the tiled plan
    sweeps_per_step = every * max(1, 10 // every) if every > 0 else 10
    roof_launches = 200
    total_sweeps = (args.warmup + args.steps + 10 * roof_launches) * sweeps_per_step
    cfg = pt.Config(w.model, w.L, w.R, w.beta, J=w.J, seed=w.seed, coupling_seed=w.coupling_seed,
                    record_every=w.record_every, max_records=total_sweeps // w.record_every)
    sim = pt.Simulation(cfg, device="cuda:0")
    if args.plan != "auto" or args.tile_planes or args.sweeps_per_launch or args.threads:
        p = sim.plan()
        mode = {"auto": p["mode"], "fused": pt.PT_PLAN_FUSED, "tiled": pt.PT_PLAN_TILED,
                "persistent": pt.PT_PLAN_PERSISTENT, "lanes": pt.PT_PLAN_LANES,
                "wave": pt.PT_PLAN_WAVE}[args.plan]
        if args.plan == "auto" and (args.tile_planes or args.sweeps_per_launch):
            mode = pt.PT_PLAN_TILED
        sim.set_plan(mode, args.tile_planes or p["tile_planes"],
                     args.sweeps_per_launch or p["sweeps_per_launch"], args.threads or p["block_threads"])
    plan = sim.plan()
    stream = sim.stream

    # warmup
    sim.run(args.warmup * sweeps_per_step, every)
    torch.cuda.synchronize()

    # timed region: exactly K steps, handed to the library as one run of the
    # schedule (as a user runs a job: the library splits it into launches;
    # fused and persistent plans run up to 4096 sweeps per launch)
    t0 = time.perf_counter()
    sim.run(args.steps * sweeps_per_step, every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    attempts = args.steps * sweeps_per_step * w.attempts_per_sweep
    value = attempts / dt

    # roofline of the sweep kernel: HIP events around single launches on the
    # library's stream (each pt_run call below is one sweep-kernel launch; with
    # whole-replica tiles a launch that ends at an exchange point is followed by
    # the exchange step's own small launch, inside the same events)
    if plan["mode"] == pt.PT_PLAN_TILED:
        per_launch = plan["sweeps_per_launch"]
        if every:
            per_launch = max(d for d in range(1, per_launch + 1) if every % d == 0)
    else:
        per_launch = 10 * sweeps_per_step  # ten steps inside one launch
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(roof_launches)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(roof_launches)]
    with torch.cuda.stream(stream):
        for i in range(roof_launches):
            starts[i].record(stream)
            sim.run(per_launch, every)
            ends[i].record(stream)
    torch.cuda.synchronize()
    durs = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    avg_ms = sum(durs) / len(durs)
    attempts_launch = per_launch * w.attempts_per_sweep
    launch_s = avg_ms * 1e-3
    achieved = SLOTS_PER_ATTEMPT * attempts_launch / launch_s / 1e12
    # algorithmic HBM bytes of one launch: every walker's packed lattice read
    # (interior plus 2 halo planes per sweep per side and tile) and written once
    tiles = -(-w.L // plan["tile_planes"]) if plan["mode"] == pt.PT_PLAN_TILED else 1
    halo_planes = 2 * 2 * per_launch * tiles if tiles > 1 else 0
    plane_bits = w.L ** (w.dim - 1)
    hbm_bytes = w.R * ((w.L + halo_planes) * plane_bits + w.L * plane_bits) / 8
    if w.dim == 3:
        hbm_bytes += 3 * w.sites / 8 * (tiles if tiles > 1 else 1)  # packed couplings, read once per tile
    split = plan["mode"] == pt.PT_PLAN_PERSISTENT and plan["tile_planes"] < w.L
    phased = w.dim == 2 and (w.L & (w.L - 1) or w.L < 8)  # sides that are not powers of two
    kernel = {pt.PT_PLAN_TILED: ("k_phased" if phased else "k_tiled_n") if w.dim == 2 else "k_tiled",
              pt.PT_PLAN_FUSED: "k_fused",
              pt.PT_PLAN_PERSISTENT: "k_persist_split" if split else "k_persist",
              pt.PT_PLAN_LANES: "k_lanes", pt.PT_PLAN_WAVE: "k_wave"}[plan["mode"]]
    traffic = measured_traffic(kernel, w.name, plan, per_launch)
    valu_insts = measured_valu_insts(kernel, w.name, plan, per_launch)
    lds_per = LDS_BYTES_PER_ATTEMPT.get("%s/%d" % (kernel, w.dim))
    lds_bytes = lds_per * attempts_launch if lds_per else None
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "Tops/s (int32 VALU lane slots)", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": traffic, "kernel": kernel,
                "slots_per_attempt": SLOTS_PER_ATTEMPT,
                "avg_launch_ms": round(avg_ms, 5), "median_launch_ms": round(durs[len(durs) // 2], 5),
                "sweeps_per_launch": per_launch,
                "attempts_per_s_in_kernel": attempts_launch / launch_s,
                # VALU instructions the kernel actually issues (SQ counters of this
                # build), as lane slots against the same peak
                "valu_insts_per_attempt": (round(valu_insts * 64 / attempts_launch, 3)
                                           if valu_insts else None),
                "issue_frac": (round(valu_insts * 64 / launch_s / 1e12 / VALU_PEAK_TOPS, 4)
                               if valu_insts else None),
                "lds_bytes_per_attempt": lds_per,
                "lds_frac": round(lds_bytes / launch_s / 1e12 / LDS_PEAK_TBPS, 4) if lds_bytes else None,
                "hbm_frac": (round(traffic / launch_s / 1e12 / HBM_PEAK_TBPS, 5) if traffic else None),
                "hbm_algorithmic_bytes_per_launch": int(hbm_bytes),
                "hbm_algorithmic_GBps": round(hbm_bytes / launch_s / 1e9, 1)}
    if split:
        # each of the P workgroups of a walker posts its two lowest and two
        # highest planes (rows in 2D) and its energy shares every sweep as 64-bit
        # tagged words, and reads as many
        parts = w.L // plan["tile_planes"]
        post_bytes = 8 * (4 * plane_bits // 32 + 2)
        roofline["boundary_post_bytes_per_launch"] = 2 * post_bytes * parts * w.R * per_launch

    if plan["mode"] in (pt.PT_PLAN_FUSED, pt.PT_PLAN_WAVE, pt.PT_PLAN_LANES):
        # One workgroup runs every walker: a sweep is a chain of dependent steps
        # (cross-lane reads, LDS round trips, barriers), far from any throughput
        # roof.  Its floor here: the same plan and schedule with a single walker,
        # whose chain is the same but contends with nothing.
        cfg1 = pt.Config(w.model, w.L, 1, w.beta[:1], J=w.J, seed=w.seed,
                         coupling_seed=w.coupling_seed, record_every=w.record_every,
                         max_records=(roof_launches + 1) * per_launch // w.record_every)
        one = pt.Simulation(cfg1, device="cuda:0")
        one.set_plan(plan["mode"], plan["tile_planes"], plan["sweeps_per_launch"], plan["block_threads"])
        one.run(per_launch, every)
        s1 = [torch.cuda.Event(enable_timing=True) for _ in range(roof_launches)]
        e1 = [torch.cuda.Event(enable_timing=True) for _ in range(roof_launches)]
        with torch.cuda.stream(one.stream):
            for i in range(roof_launches):
                s1[i].record(one.stream)
                one.run(per_launch, every)
                e1[i].record(one.stream)
        torch.cuda.synchronize()
        floor_ms = sum(a.elapsed_time(b) for a, b in zip(s1, e1)) / roof_launches
        one.close()
        us, floor_us = avg_ms * 1e3 / per_launch, floor_ms * 1e3 / per_launch
        throughput = roofline
        roofline = {"bound": "latency", "achieved": round(us, 4), "peak": round(floor_us, 4),
                    "unit": "us per sweep (lower is better)", "frac": round(floor_us / us, 4),
                    "traffic": None, "kernel": kernel,
                    "floor": "the same plan and schedule with one walker (no contention)",
                    "avg_launch_ms": throughput["avg_launch_ms"], "sweeps_per_launch": per_launch,
                    "attempts_per_s_in_kernel": throughput["attempts_per_s_in_kernel"],
                    "alu_frac": throughput["frac"]}

    if args.copy_calibration:
        a = torch.empty(64 << 20, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    obs = sim.observables(series=False)
    assert obs["sweeps_done"] == (args.warmup + args.steps) * sweeps_per_step + roof_launches * per_launch

    out = {
        "metric": "spin-flip attempts/s", "value": value, "unit": "flip attempts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": w.name, "model": "ising2d" if w.dim == 2 else "ea3d_pmJ",
                   "L": w.L, "R": w.R, "beta": [float(w.beta[0]), float(w.beta[-1])],
                   "sweeps_per_step": sweeps_per_step, "exchange_every": every,
                   "record_every": w.record_every, "seed": w.seed, "plan": plan,
                   "parallelism": "single GPU"},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        # a bounded sample: at most ~3*10^8 attempts (tens of seconds on one core)
        out["cpu_baseline"] = cpu_baseline(w, max(1, min(args.cpu_sweeps,
                                                         int(3e8 // w.attempts_per_sweep))), every)
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
