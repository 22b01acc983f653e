"""Seeded random configurations against the oracle, bit for bit.

Each case draws a model, lattice, replica count, beta ladder, field (2D), seed,
schedule (sweeps, exchange interval, record interval), a launch plan (any
mode, tile height, sweeps per launch, threads, one to eight workgroups per
walker) and whether the run goes through pt_run or the primitive pt_sweep /
pt_exchange calls.  A plan the library rejects for this shape must be rejected
with PT_EINVAL (and the automatic plan is used instead); every run must equal
the oracle's in every observable.  The cases are fixed by the generator's seed,
so a failure names a reproducible case.
"""
import numpy as np
import pytest

from gpu_common import compare, requires_gpu, say
from paper_2512_03825_amd.workloads import beta_geometric, beta_linear

pytestmark = [pytest.mark.gpu, requires_gpu]

FUSED, TILED, PERSISTENT, LANES, WAVE = 1, 2, 3, 4, 5
PT_EINVAL = -1
N_CASES = 120


def draw_case(i):
    rng = np.random.default_rng([2024, i])
    model = int(rng.random() < 0.4)
    if model == 0:
        L = int(rng.choice([8, 16, 32, 64]))
        R = int(rng.integers(2, 13))
        h = float(rng.choice([0.0, 0.0, rng.uniform(-0.2, 0.2)]))
        beta = beta_linear(0.2, 0.7, R) if rng.random() < 0.5 else beta_geometric(0.2, 0.7, R)
    else:
        L = int(rng.choice([8, 16, 32]))
        R = int(rng.integers(2, 7 if L == 32 else 10))
        h = 0.0
        beta = beta_geometric(0.4, 3.0, R)
    sweeps = int(rng.integers(5, 41))
    every = int(rng.choice([0, 1, 2, 3, 5]))
    rec = int(rng.choice([0, 1, 2, 3]))
    # 3D cases lean to the persistent plans (one or two workgroups per walker)
    modes = [FUSED, TILED, PERSISTENT, LANES, WAVE] if model == 0 else [FUSED, TILED, PERSISTENT, PERSISTENT]
    mode = int(rng.choice(modes))
    threads = int(rng.integers(1, 17)) * 64
    plan = dict(mode=mode, block_threads=threads)
    if mode == TILED:
        plan.update(tile_planes=int(rng.integers(1, L + 1)), sweeps_per_launch=int(rng.integers(1, 17)))
    elif mode == PERSISTENT:
        plan.update(tile_planes=int(rng.choice([L, L // 2, L // 2, L // 4, L // 8])))
    primitive = bool(rng.random() < 0.3)
    return dict(model=model, L=L, R=R, h=h, beta=beta, seed=int(rng.integers(1, 1 << 30)),
                coupling_seed=int(rng.integers(1, 1 << 30)), sweeps=sweeps, every=every, rec=rec,
                plan=plan, primitive=primitive)


def draw_even_side_case(i):
    """2D cases on even sides that are not powers of two (the phased rows) and
    on larger powers of two (the split plans, with their handshakes overlapped
    between exchange steps), any plan, up to 16 sweeps per launch."""
    rng = np.random.default_rng([2025, i])
    L = int(rng.choice([10, 12, 14, 18, 20, 22, 26, 30, 36, 46, 50, 60, 62, 72, 100, 64, 128]))
    R = int(rng.integers(2, 13))
    h = float(rng.choice([0.0, 0.0, rng.uniform(-0.2, 0.2)]))
    beta = beta_linear(0.2, 0.7, R) if rng.random() < 0.5 else beta_geometric(0.2, 0.7, R)
    sweeps = int(rng.integers(5, 41))
    every = int(rng.choice([0, 1, 2, 3, 5, 7]))
    rec = int(rng.choice([0, 1, 2, 3]))
    mode = int(rng.choice([TILED, TILED, PERSISTENT, PERSISTENT, FUSED]))
    plan = dict(mode=mode, block_threads=int(rng.integers(1, 17)) * 64)
    if mode == TILED:
        plan.update(tile_planes=int(rng.choice([L, L, max(1, L // 2), int(rng.integers(1, L + 1))])),
                    sweeps_per_launch=int(rng.integers(1, 17)))
    elif mode == PERSISTENT:
        plan.update(tile_planes=int(rng.choice([L, L // 2, L // 4, L // 8])))
    primitive = bool(rng.random() < 0.3)
    return dict(model=0, L=L, R=R, h=h, beta=beta, seed=int(rng.integers(1, 1 << 30)),
                coupling_seed=int(rng.integers(1, 1 << 30)), sweeps=sweeps, every=every, rec=rec,
                plan=plan, primitive=primitive)


@pytest.mark.parametrize("i", range(N_CASES))
def test_random_case_matches_oracle(oracle_mod, i):
    run_random_case(oracle_mod, "fuzz %d" % i, draw_case(i))


@pytest.mark.parametrize("i", range(60))
def test_random_even_side_case_matches_oracle(oracle_mod, i):
    run_random_case(oracle_mod, "fuzz-even %d" % i, draw_even_side_case(i))


def run_random_case(oracle_mod, name, c):
    from paper_2512_03825_amd import pt
    tag = "%s: model %d L %d R %d h %.3f sweeps %d every %d rec %d plan %s primitive %s" % (
        name, c["model"], c["L"], c["R"], c["h"], c["sweeps"], c["every"], c["rec"], c["plan"],
        c["primitive"])
    say(tag)
    nrec = c["sweeps"] // c["rec"] if c["rec"] else 0
    kw = dict(h=c["h"], seed=c["seed"], coupling_seed=c["coupling_seed"], record_every=c["rec"],
              max_records=nrec)
    sim = pt.Simulation(pt.Config(c["model"], c["L"], c["R"], c["beta"], **kw))
    try:
        sim.set_plan(**c["plan"])
    except pt.PTError as err:
        assert err.status == PT_EINVAL, tag
        say("  plan rejected for this shape; automatic plan", sim.plan())
    orc = oracle_mod.Oracle(c["model"], c["L"], c["R"], c["beta"], **kw)
    if c["primitive"]:
        done = 0
        while done < c["sweeps"]:
            n = min(c["every"], c["sweeps"] - done) if c["every"] else c["sweeps"] - done
            sim.sweep(n)
            orc.sweep(n)
            done += n
            if c["every"] and done % c["every"] == 0:
                sim.exchange()
                orc.exchange()
    else:
        sim.run(c["sweeps"], c["every"])
        orc.run(c["sweeps"], c["every"])
    compare(sim, orc, tag)
    sim.close()
