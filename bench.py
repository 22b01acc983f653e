"""Throughput benchmark: parallel-tempering Metropolis on one MI355X.

Workload (default): 2D Ising 1024x1024, J = 1, h = 0, R = 64 replicas with beta
linear in [0.30, 0.55], spins drawn from seed 2; E_int and M reduced and
recorded after every sweep; one replica-exchange step every 10 sweeps.
A step is one interval of that schedule (10 checkerboard sweeps of all 64
replicas + their records + one exchange step, i.e. 6.7e8 flip attempts); the
full run of the workload is 1000 steps (10^4 sweeps).

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
# slots per second for 32-bit integer operations.  On gfx950 the 32x32->64
# multiply-add (v_mad_u64_u32) and the three-input XOR (v_bitop3_b32) both issue
# at that full rate (measured: 34.8e12 and 33.4e12 lane ops/s in dependent-free
# probe loops).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic VALU slots per flip attempt: a quarter of one Philox4x32-10 block
# (20 multiplies + 20 three-input XORs = 40 slots per block of 4 draws) plus the
# stencil and decision (2D: 10 -- neighbour sum, spin product, class, threshold
# compare, conditional flip, E/M update; 3D +-J: 20 with the six couplings).
SLOTS_PER_ATTEMPT = {2: 10 + 10, 3: 10 + 20}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ising2d_L1024_R64")
    ap.add_argument("--tile-planes", type=int, default=0)
    ap.add_argument("--sweeps-per-launch", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=4)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 64 MiB device-to-device copy (a kernel of known "
                         "traffic, to scale HBM counters)")
    return ap.parse_args()


def cpu_baseline(w, sweeps):
    """The CPU oracle, as it stands, on a bounded prefix of the same workload."""
    import oracle
    o = oracle.Oracle(w.model, w.L, w.R, w.beta, seed=w.seed, coupling_seed=w.coupling_seed)
    t0 = time.perf_counter()
    o.run(sweeps, w.exchange_every)
    dt = time.perf_counter() - t0
    attempts = sweeps * w.attempts_per_sweep
    return {"value": attempts / dt, "unit": "flip attempts/s", "cores": 1, "kind": "oracle",
            "sample": "%s: first %d sweeps after initialisation (%.3g flip attempts, %.1f s, "
                      "single thread)" % (w.name, sweeps, attempts, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(the path would shard by temperature slots, see the design notes)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2512_03825_amd import pt
    from paper_2512_03825_amd.workloads import HOT_PATH

    w = HOT_PATH[args.workload]
    torch.cuda.set_device(0)
    every = w.exchange_every
    sweeps_per_step = every if every > 0 else 10
    roof_launches = 200
    total_sweeps = (args.warmup + args.steps) * sweeps_per_step + roof_launches * 8
    cfg = pt.Config(w.model, w.L, w.R, w.beta, J=w.J, seed=w.seed, coupling_seed=w.coupling_seed,
                    record_every=w.record_every, max_records=total_sweeps // w.record_every)
    sim = pt.Simulation(cfg, device="cuda:0")
    if args.tile_planes or args.sweeps_per_launch or args.threads:
        p = sim.plan()
        sim.set_plan(pt.PT_PLAN_TILED, args.tile_planes or p["tile_planes"],
                     args.sweeps_per_launch or p["sweeps_per_launch"], args.threads or p["block_threads"])
    plan = sim.plan()
    stream = sim.stream

    # warmup
    for _ in range(args.warmup):
        sim.run(sweeps_per_step, every)
    torch.cuda.synchronize()

    # timed region: exactly K steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sim.run(sweeps_per_step, every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    attempts = args.steps * sweeps_per_step * w.attempts_per_sweep
    value = attempts / dt

    # roofline of the sweep kernel: HIP events around single launches on the
    # library's stream (each pt_run call below is exactly one kernel launch)
    per_launch = plan["sweeps_per_launch"] if plan["mode"] == pt.PT_PLAN_TILED else 1
    if every:
        per_launch = max(d for d in range(1, per_launch + 1) if every % d == 0)
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
    slots = SLOTS_PER_ATTEMPT[w.dim] * per_launch * w.attempts_per_sweep
    achieved = slots / (avg_ms * 1e-3) / 1e12
    # algorithmic HBM bytes of one launch: every walker's packed lattice read
    # (interior plus 2 halo planes per sweep per side and tile) and written once
    tiles = -(-w.L // plan["tile_planes"]) if plan["mode"] == pt.PT_PLAN_TILED else 1
    halo_planes = 2 * 2 * per_launch * tiles if tiles > 1 else 0
    plane_bits = w.L ** (w.dim - 1)
    hbm_bytes = w.R * ((w.L + halo_planes) * plane_bits + w.L * plane_bits) / 8
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "Tops/s (int32 VALU lane slots)", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": None, "kernel": "k_tiled" if plan["mode"] == pt.PT_PLAN_TILED else "k_fused",
                "slots_per_attempt": SLOTS_PER_ATTEMPT[w.dim],
                "avg_launch_ms": round(avg_ms, 5), "median_launch_ms": round(durs[len(durs) // 2], 5),
                "sweeps_per_launch": per_launch,
                "attempts_per_s_in_kernel": per_launch * w.attempts_per_sweep / (avg_ms * 1e-3),
                "hbm_algorithmic_bytes_per_launch": int(hbm_bytes),
                "hbm_algorithmic_GBps": round(hbm_bytes / (avg_ms * 1e-3) / 1e9, 1)}

    if args.copy_calibration:
        a = torch.empty(64 << 20, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    obs = sim.observables(series=False)
    assert obs["sweeps_done"] == total_sweeps - roof_launches * 8 + roof_launches * per_launch

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
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sweeps)
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
