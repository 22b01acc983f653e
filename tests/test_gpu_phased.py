"""2D lattices whose side is even but not a power of two (rows that are not a
whole number of the 8-site groups one Philox block serves): the paper's own
300 x 300 lattice (Sec. 4.2) and sides from 4 up, on the phased whole-replica
kernel, compared bit for bit with the oracle (spins, E/M series, walker map,
swap counts) over schedules with and without exchanges, fields, and
sweeps-per-launch counts and block sizes across what the plan allows."""
import numpy as np
import pytest

from gpu_common import compare, make_gpu, make_oracle, requires_gpu, say
from paper_2512_03825_amd.workloads import beta_geometric, beta_linear, paper_shape

pytestmark = [pytest.mark.gpu, requires_gpu]

CASES = [
    # L, R, sweeps, exchange_every, h, plan (None = automatic)
    (4, 3, 21, 1, 0.0, None),
    (6, 4, 17, 3, 0.07, None),
    (10, 2, 25, 5, 0.0, None),
    (12, 5, 20, 2, 0.0, None),
    (12, 8, 16, 4, -0.05, dict(mode=2, tile_planes=12, sweeps_per_launch=3, block_threads=64)),
    (14, 3, 19, 0, 0.0, None),
    (20, 6, 30, 5, 0.0, None),
    (22, 2, 15, 1, 0.03, dict(mode=2, tile_planes=22, sweeps_per_launch=1, block_threads=128)),
    (24, 4, 18, 6, 0.0, None),
    (36, 3, 14, 7, 0.0, dict(mode=2, tile_planes=64, sweeps_per_launch=5, block_threads=1024)),
    (44, 7, 12, 3, 0.0, None),
    (60, 4, 11, 2, 0.0, None),
    (100, 5, 10, 5, 0.02, dict(mode=2, tile_planes=100, sweeps_per_launch=8, block_threads=512)),
    (300, 4, 9, 3, 0.0, None),
    (300, 3, 8, 4, 0.0, dict(mode=2, tile_planes=300, sweeps_per_launch=2, block_threads=1024)),
    (520, 2, 6, 3, 0.0, None),
    # rows whose last dword is past some rows' end (L = 46: phases 0..6), and
    # runs of 16 sweeps per launch with a ragged last launch
    (46, 3, 19, 4, 0.0, None),
    (50, 4, 35, 0, 0.05, None),
    (100, 5, 40, 8, 0.02, dict(mode=2, tile_planes=100, sweeps_per_launch=16, block_threads=512)),
    (300, 3, 37, 0, 0.0, None),
]


@pytest.mark.parametrize("L, R, sweeps, every, h, plan", CASES)
def test_phased_rows_match_oracle(oracle_mod, pt, L, R, sweeps, every, h, plan):
    beta = beta_linear(0.30, 0.55, R)
    say("phased", "L", L, "R", R, "sweeps", sweeps, "every", every, "h", h, "plan", plan)
    cfg = pt.Config(0, L, R, beta, h=h, seed=11 + L, record_every=1, max_records=sweeps)
    sim = pt.Simulation(cfg)
    if plan is not None:
        sim.set_plan(**plan)
    p = sim.plan()
    assert p["mode"] == 2 and p["tile_planes"] >= L, p
    sim.run(sweeps, every)
    orc = oracle_mod.Oracle(0, L, R, beta, h=h, seed=11 + L, record_every=1, max_records=sweeps)
    orc.run(sweeps, every)
    compare(sim, orc, "phased L %d R %d" % (L, R))
    sim.close()


def test_phased_primitive_calls_and_uploads(oracle_mod, pt):
    """pt_sweep / pt_exchange intervals and uploaded spins on a 30 x 30 lattice."""
    L, R = 30, 4
    beta = beta_geometric(0.2, 0.7, R)
    rng = np.random.default_rng(3)
    s0 = np.where(rng.random((R, L * L)) < 0.3, -1, 1).astype(np.int8)
    sim = make_gpu(pt, 0, L, R, beta, seed=5, init_spins=s0, record_every=2, max_records=20)
    orc = make_oracle(oracle_mod, 0, L, R, beta, seed=5, init_spins=s0, record_every=2, max_records=20)
    for n in (3, 1, 4, 2):
        sim.sweep(n)
        sim.exchange()
        orc.sweep(n)
        orc.exchange()
    compare(sim, orc, "phased primitives")
    sim.close()


def test_phased_plans_are_checked(pt):
    cfg = pt.Config(0, 300, 2, np.array([0.4, 0.5]))
    sim = pt.Simulation(cfg)
    for bad in (dict(mode=1, block_threads=256), dict(mode=3, tile_planes=300, block_threads=1024),
                dict(mode=2, tile_planes=150, sweeps_per_launch=2, block_threads=256),
                dict(mode=5)):
        with pytest.raises(pt.PTError, match="not a power of two"):
            sim.set_plan(**bad)
    sim.close()


def test_paper_shape_300_matches_oracle(oracle_mod, pt):
    """The paper's speed-up shape itself (Sec. 4.2): 300 x 300, 1500 replicas on
    its ladder T_k = 1 + 3k/R (Sec. 3), no swaps, its run length of 3*10^5
    attempts per replica (4 sweeps), in the automatic plan bench.py times."""
    w = paper_shape(300)
    assert (w.L, w.R, w.sweeps, w.exchange_every) == (300, 1500, 4, 0)
    say("paper shape", w.name, "sweeps", w.sweeps)
    cfg = pt.Config(w.model, w.L, w.R, w.beta, seed=w.seed, record_every=1, max_records=w.sweeps)
    sim = pt.Simulation(cfg)
    say("plan", sim.plan())
    sim.run(w.sweeps, w.exchange_every)
    orc = oracle_mod.Oracle(w.model, w.L, w.R, w.beta, seed=w.seed, record_every=1, max_records=w.sweeps)
    orc.run(w.sweeps, w.exchange_every)
    compare(sim, orc, w.name)
    sim.close()


def test_paper_shape_300_with_swaps_matches_oracle(oracle_mod, pt):
    """The paper's shape with an exchange after every sweep (its own swap
    intervals are shorter than a sweep of this lattice): one-sweep launches of
    whole replicas, each followed by the exchange step as a launch of its own
    over all 750 pairs."""
    w = paper_shape(300)
    sweeps = 3
    say("paper shape with swaps", w.name, "sweeps", sweeps)
    cfg = pt.Config(w.model, w.L, w.R, w.beta, seed=w.seed, record_every=1, max_records=sweeps)
    sim = pt.Simulation(cfg)
    sim.run(sweeps, 1)
    orc = oracle_mod.Oracle(w.model, w.L, w.R, w.beta, seed=w.seed, record_every=1, max_records=sweeps)
    orc.run(sweeps, 1)
    obs = compare(sim, orc, w.name + " every sweep")
    assert obs["swap_acc"].sum() > 0
    sim.close()


@pytest.fixture(scope="module")
def pt():
    from paper_2512_03825_amd import pt as _pt
    return _pt
