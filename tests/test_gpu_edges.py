"""Degenerate and extreme configurations against the oracle, bit for bit.

- one replica (no exchange pair ever exists; exchange steps still count), in
  every plan that accepts it, 2D and 3D (the split persistent plan included);
- the largest replica count (R = 4096) and the lanes plan's largest (R = 1024);
- a run of zero sweeps (the state after initialisation), then a real run;
- an exchange interval longer than the run (no exchange step happens);
- beta far above the ordering temperature from the all-up state: every flip is
  rejected (ground-state energy -2N, M = N, exactly), which also pins the
  thresholds' saturated end.
"""
import numpy as np
import pytest

from gpu_common import compare, make_gpu, make_oracle, requires_gpu, say
from paper_2512_03825_amd.workloads import beta_geometric, beta_linear

pytestmark = [pytest.mark.gpu, requires_gpu]

FUSED, TILED, PERSISTENT, LANES, WAVE = 1, 2, 3, 4, 5


@pytest.fixture(scope="module")
def pt():
    from paper_2512_03825_amd import pt as _pt
    return _pt


def run_both(pt, oracle_mod, model, L, R, beta, sweeps, every, plan=None, rec=1, init_spins=None,
             tag=""):
    say("case", tag, "model", model, "L", L, "R", R, "sweeps", sweeps, "every", every, "plan", plan)
    nrec = sweeps // rec if rec else 0
    sim = make_gpu(pt, model, L, R, beta, 41, 7, init_spins, None, rec, nrec, plan)
    orc = make_oracle(oracle_mod, model, L, R, beta, 41, 7, init_spins, None, rec, nrec)
    sim.run(sweeps, every)
    orc.run(sweeps, every)
    obs = compare(sim, orc, tag)
    sim.close()
    return obs


@pytest.mark.parametrize("model, L, plan", [
    (0, 32, None),
    (0, 32, dict(mode=FUSED, block_threads=128)),
    (0, 64, dict(mode=TILED, tile_planes=16, sweeps_per_launch=3, block_threads=256)),
    (0, 32, dict(mode=PERSISTENT, block_threads=256)),
    (0, 16, dict(mode=LANES)),
    (0, 16, dict(mode=WAVE)),
    (1, 16, None),
    (1, 32, dict(mode=PERSISTENT, tile_planes=16, block_threads=512)),
])
def test_single_replica(pt, oracle_mod, model, L, plan):
    beta = np.array([0.6 if model == 1 else 0.4])
    obs = run_both(pt, oracle_mod, model, L, 1, beta, 30, 1, plan=plan, tag="R=1")
    assert obs["exchanges_done"] == 30 and obs["swap_att"].sum() == 0


def test_largest_replica_count(pt, oracle_mod):
    run_both(pt, oracle_mod, 0, 8, 4096, beta_linear(0.1, 0.9, 4096), 12, 3, tag="R=4096")


def test_lanes_plan_largest_replica_count(pt, oracle_mod):
    run_both(pt, oracle_mod, 0, 8, 1024, beta_linear(0.1, 0.9, 1024), 10, 2, plan=dict(mode=LANES),
             tag="lanes R=1024")


@pytest.mark.parametrize("model, L, R", [(0, 32, 6), (1, 8, 5)])
def test_zero_sweeps_then_a_run(pt, oracle_mod, model, L, R):
    beta = beta_geometric(0.2, 0.6, R) if model == 0 else beta_geometric(0.5, 3.0, R)
    sim = make_gpu(pt, model, L, R, beta, 43, 9, None, None, 1, 20)
    orc = make_oracle(oracle_mod, model, L, R, beta, 43, 9, None, None, 1, 20)
    sim.run(0, 5)
    obs = compare(sim, orc, "zero sweeps")
    assert obs["sweeps_done"] == 0 and obs["n_records"] == 0
    sim.run(20, 5)
    orc.run(20, 5)
    compare(sim, orc, "after zero sweeps")
    sim.close()


def test_interval_longer_than_the_run(pt, oracle_mod):
    obs = run_both(pt, oracle_mod, 0, 32, 6, beta_linear(0.3, 0.5, 6), 30, 100, tag="every 100")
    assert obs["exchanges_done"] == 0 and obs["swap_att"].sum() == 0


@pytest.mark.parametrize("plan", [None, dict(mode=TILED, tile_planes=8, sweeps_per_launch=2,
                                                 block_threads=256)])
def test_ordered_state_at_large_beta(pt, oracle_mod, plan):
    L, R = 32, 4
    N = L * L
    up = np.ones((R, N), np.int8)
    obs = run_both(pt, oracle_mod, 0, L, R, np.full(R, 20.0), 25, 5, plan=plan, init_spins=up,
                   tag="beta 20 from all up")
    assert np.all(obs["E_series"] == -2 * N) and np.all(obs["M_series"] == N)
    assert np.all(obs["spins"] == 1)


@pytest.mark.parametrize("every", [0, 2])
def test_paper_shape_ladder_at_reduced_size(pt, oracle_mod, every):
    """1500 replicas on the paper's temperature ladder T_k = 1 + 3k/R, on a
    32 x 32 lattice (the bench runs the same ladder at 256^2 and 512^2)."""
    from paper_2512_03825_amd.workloads import paper_shape
    beta = paper_shape(256).beta
    run_both(pt, oracle_mod, 0, 32, 1500, beta, 6, every, tag="paper ladder R=1500")


def test_auto_plans_of_the_bench_workloads(pt):
    """The decompositions the measurements describe are the ones the automatic
    plan picks for the benchmarked workloads."""
    from paper_2512_03825_amd.workloads import WORKLOADS
    want = {
        "ising2d_L16_R8": dict(mode=WAVE, block_threads=256),
        "ising2d_L1024_R64": dict(mode=PERSISTENT, tile_planes=256, block_threads=1024),
        "ea3d_L32_R128": dict(mode=PERSISTENT, tile_planes=16, block_threads=512),
        "paper_shape_L256_R1500": dict(mode=TILED, tile_planes=256, sweeps_per_launch=16,
                                       block_threads=256),
        "paper_shape_L512_R1500": dict(mode=TILED, tile_planes=512, sweeps_per_launch=16,
                                       block_threads=1024),
        "paper_shape_L300_R1500": dict(mode=TILED, tile_planes=300, sweeps_per_launch=16,
                                       block_threads=512),
    }
    for name, plan in want.items():
        w = WORKLOADS[name]
        sim = pt.Simulation(pt.Config(w.model, w.L, w.R, w.beta, seed=w.seed,
                                      coupling_seed=w.coupling_seed))
        got = sim.plan()
        sim.close()
        say("auto plan", name, got)
        assert all(got[k] == v for k, v in plan.items()), (name, got)
