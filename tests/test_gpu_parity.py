"""GPU library vs CPU oracle, bit for bit, through the C ABI.

Every case runs the same seeded configuration on both sides and compares all
spins of all slots, the walker map, the E/M record series, the current E and M,
and the swap attempt/accept counts.  Plans (fused, tiled with whole-replica or
halo tiles, ragged last tiles, 1..4 sweeps per launch, 64..1024 threads) must
all give the identical result, which doubles as the race detector.
"""
import numpy as np
import pytest

from gpu_common import compare, make_gpu, make_oracle, requires_gpu, say
from paper_2512_03825_amd.workloads import beta_geometric, beta_linear, ising16

pytestmark = [pytest.mark.gpu, requires_gpu]

FUSED, TILED, PERSISTENT, LANES, WAVE = 1, 2, 3, 4, 5


@pytest.fixture(scope="module")
def pt():
    from paper_2512_03825_amd import pt as _pt
    return _pt


def run_case(pt, oracle_mod, model, L, R, beta, seed, sweeps, every, record_every=1, plan=None,
             coupling_seed=None, init_spins=None, couplings=None, split=False, tag=""):
    say("case", tag, "model", model, "L", L, "R", R, "sweeps", sweeps, "every", every, "plan", plan)
    rec = sweeps // record_every if record_every else 0
    sim = make_gpu(pt, model, L, R, beta, seed, coupling_seed, init_spins, couplings,
                   record_every, rec, plan)
    orc = make_oracle(oracle_mod, model, L, R, beta, seed, coupling_seed, init_spins, couplings,
                      record_every, rec)
    if split:
        # the primitive calls: pt_sweep intervals and pt_exchange steps
        done = 0
        while done < sweeps:
            n = min(every, sweeps - done) if every else sweeps - done
            sim.sweep(n)
            orc.sweep(n)
            done += n
            if every and done % every == 0:
                sim.exchange()
                orc.exchange()
    else:
        sim.run(sweeps, every)
        orc.run(sweeps, every)
    compare(sim, orc, tag)
    return sim, orc


def test_ising16_full_run_auto_plan(pt, oracle_mod):
    """2D Ising 16x16, R = 8, 1000 sweeps, exchange every 10: the whole run, default plan."""
    w = ising16()
    sim, orc = run_case(pt, oracle_mod, 0, w.L, w.R, w.beta, w.seed, w.sweeps, w.exchange_every,
                        tag="ising16")
    assert sim.plan()["mode"] == WAVE
    assert orc.swaps()[1].sum() > 0  # swaps really happen


@pytest.mark.parametrize("plan", [
    dict(mode=TILED, tile_planes=16, sweeps_per_launch=1, block_threads=64),    # whole replica
    dict(mode=TILED, tile_planes=16, sweeps_per_launch=3, block_threads=256),
    dict(mode=TILED, tile_planes=32, sweeps_per_launch=8, block_threads=1024),
    dict(mode=FUSED, block_threads=64),
    dict(mode=FUSED, block_threads=1024),
    dict(mode=LANES),                                                           # one walker per lane
    dict(mode=WAVE),                                                            # walkers in wavefronts
])
def test_ising16_every_plan_is_identical(pt, oracle_mod, plan):
    w = ising16()
    run_case(pt, oracle_mod, 0, w.L, w.R, w.beta, w.seed, 200, w.exchange_every, plan=plan,
             tag="ising16-plan")


@pytest.mark.parametrize("plan", [
    dict(mode=TILED, tile_planes=4, sweeps_per_launch=1, block_threads=64),     # halo tiles
    dict(mode=TILED, tile_planes=5, sweeps_per_launch=2, block_threads=128),    # ragged last tile
    dict(mode=TILED, tile_planes=3, sweeps_per_launch=4, block_threads=1024),
    dict(mode=TILED, tile_planes=8, sweeps_per_launch=3, block_threads=256),
    dict(mode=TILED, tile_planes=32, sweeps_per_launch=5, block_threads=512),   # whole replica
    dict(mode=FUSED, block_threads=256),
])
def test_ising32_halo_plans(pt, oracle_mod, plan):
    """Halo tiles (2 rows per sweep per side), ragged tails, 1..5 sweeps per launch."""
    beta = beta_geometric(0.20, 0.60, 8)
    run_case(pt, oracle_mod, 0, 32, 8, beta, 13, 120, 10, plan=plan, tag="ising32-plan")


@pytest.mark.parametrize("plan", [
    None,
    dict(mode=TILED, tile_planes=64, sweeps_per_launch=2, block_threads=256),
    dict(mode=TILED, tile_planes=8, sweeps_per_launch=1, block_threads=256),
    dict(mode=TILED, tile_planes=13, sweeps_per_launch=3, block_threads=512),
])
def test_ising64_odd_R(pt, oracle_mod, plan):
    """Several tiles, a ragged tail, odd R (the top slot sits out every other step)."""
    beta = beta_linear(0.30, 0.55, 5)
    run_case(pt, oracle_mod, 0, 64, 5, beta, 7, 60, 3, record_every=2, plan=plan, tag="ising64")


@pytest.mark.parametrize("plan", [
    None,
    dict(mode=FUSED, block_threads=256),
    dict(mode=TILED, tile_planes=8, sweeps_per_launch=1, block_threads=256),
    dict(mode=TILED, tile_planes=2, sweeps_per_launch=1, block_threads=128),
    dict(mode=TILED, tile_planes=3, sweeps_per_launch=2, block_threads=256),
])
def test_ea8(pt, oracle_mod, plan):
    beta = beta_geometric(0.5, 3.0, 6)
    run_case(pt, oracle_mod, 1, 8, 6, beta, 3, 50, 1, plan=plan, coupling_seed=3, tag="ea8")


@pytest.mark.parametrize("plan", [
    None,
    dict(mode=TILED, tile_planes=4, sweeps_per_launch=2, block_threads=256),
    dict(mode=TILED, tile_planes=16, sweeps_per_launch=1, block_threads=512),
])
def test_ea16(pt, oracle_mod, plan):
    beta = beta_geometric(0.5, 3.0, 4)
    run_case(pt, oracle_mod, 1, 16, 4, beta, 3, 20, 1, plan=plan, coupling_seed=5, tag="ea16")


@pytest.mark.parametrize("model, L, R, every, threads", [
    (0, 16, 8, 10, 256),    # the 16x16 workload's shape
    (0, 32, 7, 1, 128),     # odd R, exchange every sweep
    (0, 64, 12, 3, 512),
    (1, 8, 6, 1, 256),
    (1, 16, 5, 2, 1024),
    (1, 32, 4, 1, 1024),    # the EA workload's lattice
])
def test_persistent_plan(pt, oracle_mod, model, L, R, every, threads):
    """One workgroup per walker for the whole run; pairwise exchange decisions."""
    beta = beta_geometric(0.5, 3.0, R) if model == 1 else beta_geometric(0.2, 0.6, R)
    plan = dict(mode=PERSISTENT, block_threads=threads)
    run_case(pt, oracle_mod, model, L, R, beta, 17, 40, every, plan=plan, coupling_seed=4,
             tag="persist")
    run_case(pt, oracle_mod, model, L, R, beta, 17, 24, every, plan=plan, coupling_seed=4,
             split=True, tag="persist-split")


@pytest.mark.parametrize("L, R, every, rec, threads", [
    (16, 5, 2, 1, 512),     # one group per item
    (16, 6, 1, 2, 1024),
    (32, 4, 1, 1, 1024),    # the EA workload's lattice, two groups per item
    (32, 7, 3, 1, 512),     # four groups per item, odd R
    (32, 9, 1, 3, 768),     # more threads than a pass has items in the last rounds
    (32, 5, 0, 1, 256),     # no exchange steps: boundary posts only
    (32, 6, 1, 1, 576),     # one item per computing thread: counts taken during the handshake
    (32, 7, 2, 2, 576),
    (16, 5, 1, 1, 192),     # the same at L = 16 (two groups per item)
    (16, 4, 0, 3, 192),
])
def test_split_persistent_plan(pt, oracle_mod, L, R, every, rec, threads):
    """3D walkers split over two co-resident workgroups of L/2 z-planes each."""
    beta = beta_geometric(0.5, 3.0, R)
    plan = dict(mode=PERSISTENT, tile_planes=L // 2, block_threads=threads)
    sim, _ = run_case(pt, oracle_mod, 1, L, R, beta, 23, 36, every, record_every=rec, plan=plan,
                      coupling_seed=6, tag="persist-2")
    assert sim.plan()["tile_planes"] == L // 2
    run_case(pt, oracle_mod, 1, L, R, beta, 23, 18, every, record_every=rec, plan=plan,
             coupling_seed=6, split=True, tag="persist-2-split")


@pytest.mark.parametrize("L, R, every, rec, threads, parts", [
    (64, 4, 1, 1, 256, 2),
    (64, 3, 3, 2, 256, 4),      # odd R
    (64, 5, 1, 1, 512, 8),      # eight rows per part
    (128, 4, 2, 1, 512, 4),
    (256, 3, 0, 1, 1024, 8),    # no exchange steps: boundary posts only
    (1024, 2, 1, 1, 1024, 4),   # the 1024^2 workload's decomposition
    (1024, 3, 5, 2, 1024, 4),   # handshakes overlapped with the next sweep between exchanges
])
def test_split_persistent_plan_2d(pt, oracle_mod, L, R, every, rec, threads, parts):
    """2D walkers split over P co-resident workgroups of L/P rows each."""
    beta = beta_geometric(0.2, 0.6, R)
    plan = dict(mode=PERSISTENT, tile_planes=L // parts, block_threads=threads)
    sweeps = 24 if L < 1024 else 12
    sim, _ = run_case(pt, oracle_mod, 0, L, R, beta, 29, sweeps, every, record_every=rec,
                      plan=plan, tag="persist-2d-%d" % parts)
    assert sim.plan()["tile_planes"] == L // parts
    run_case(pt, oracle_mod, 0, L, R, beta, 29, sweeps // 2, every, record_every=rec, plan=plan,
             split=True, tag="persist-2d-%d-split" % parts)


@pytest.mark.parametrize("L, R, every, h, parts, threads, split", [
    (32, 6, 1, 0.1, 1, 256, False),      # one workgroup per walker
    (64, 5, 3, -0.05, 1, 512, True),
    (64, 4, 1, 0.1, 2, 256, False),      # rows split over P workgroups
    (128, 5, 2, -0.08, 4, 512, True),
    (256, 3, 1, 0.05, 8, 1024, False),
])
def test_persistent_plans_with_field(pt, oracle_mod, L, R, every, h, parts, threads, split):
    """2D with h != 0: the persistent plans' pairwise exchange decisions include
    the field factor (both walkers' magnetisations through the mailboxes).  The
    ladder is narrow enough that swaps are accepted in every case."""
    beta = beta_linear(0.40, 0.40 + 2.0 / L, R)
    sweeps = 24
    tag = "persist field L%d R%d P%d h%.2f" % (L, R, parts, h)
    say("case", tag, "every", every, "split", split)
    cfg = pt.Config(0, L, R, beta, h=h, seed=31, stream_id=2, record_every=1, max_records=sweeps)
    sim = pt.Simulation(cfg)
    sim.set_plan(PERSISTENT, tile_planes=L // parts, block_threads=threads)
    assert sim.plan()["mode"] == PERSISTENT and sim.plan()["tile_planes"] == L // parts
    orc = oracle_mod.Oracle(0, L, R, beta, h=h, seed=31, stream_id=2, record_every=1,
                            max_records=sweeps)
    if split:
        for _ in range(sweeps // every):
            sim.sweep(every)
            sim.exchange()
            orc.sweep(every)
            orc.exchange()
    else:
        sim.run(sweeps, every)
        orc.run(sweeps, every)
    obs = compare(sim, orc, tag)
    assert obs["swap_acc"].sum() > 0


def test_split_persistent_plan_rejects_other_shapes(pt):
    for model, L in ((0, 32), (1, 8), (1, 64)):  # lattices too small or too large to split
        cfg = pt.Config(model, L, 4, beta_geometric(0.5, 3.0, 4), seed=1)
        sim = pt.Simulation(cfg)
        with pytest.raises(pt.PTError):
            sim.set_plan(PERSISTENT, tile_planes=L // 2, block_threads=256)
        with pytest.raises(pt.PTError):
            sim.set_plan(PERSISTENT, tile_planes=3, block_threads=256)
        sim.close()
    # 2D: parts of fewer than 8 rows, a non-power-of-two part count, a lattice too large
    for L, tp in ((64, 4), (64, 24), (2048, 256)):
        sim = pt.Simulation(pt.Config(0, L, 2, beta_geometric(0.2, 0.6, 2), seed=1))
        with pytest.raises(pt.PTError):
            sim.set_plan(PERSISTENT, tile_planes=tp, block_threads=256)
        sim.close()


@pytest.mark.parametrize("model, L, R, plan, every", [
    (1, 32, 6, dict(mode=PERSISTENT, tile_planes=16, block_threads=512), 1),   # two workgroups per walker
    (1, 16, 5, dict(mode=PERSISTENT, tile_planes=16, block_threads=256), 1),   # one per walker
    (0, 32, 8, dict(mode=PERSISTENT, block_threads=256), 1),
    (0, 64, 4, dict(mode=PERSISTENT, tile_planes=16, block_threads=256), 1),   # 2D, four per walker
    (0, 128, 3, dict(mode=PERSISTENT, tile_planes=64, block_threads=512), 1),  # 2D, two per walker
    # a handshake overlapped with the next sweep gives up (no exchange step, or one every 5)
    (0, 64, 4, dict(mode=PERSISTENT, tile_planes=16, block_threads=256), 0),
    (0, 128, 3, dict(mode=PERSISTENT, tile_planes=32, block_threads=1024), 5),
])
def test_persistent_wait_bound_stops_the_launch(pt, oracle_mod, model, L, R, plan, every):
    """A wait limit of 0 makes every bounded wait give up at once: the launch
    ends early (every workgroup leaves its loop), the next observables call
    reports PT_EDEVICE and the context stays poisoned; a new context then runs
    normally."""
    PT_EDEVICE, PT_ESTATE = -3, -4
    beta = beta_geometric(0.5, 3.0, R) if model == 1 else beta_geometric(0.2, 0.6, R)
    sim = make_gpu(pt, model, L, R, beta, 29, 8, None, None, 1, 10, plan)
    say("case wait bound", model, L, R, plan, "every", every)
    sim.set_wait_limit(0)
    sim.run(10, every)
    with pytest.raises(pt.PTError) as err:
        sim.observables()
    assert err.value.status == PT_EDEVICE
    with pytest.raises(pt.PTError) as err:
        sim.run(1, 1)
    assert err.value.status == PT_ESTATE
    sim.close()
    run_case(pt, oracle_mod, model, L, R, beta, 29, 6, 1, plan=plan, coupling_seed=8,
             tag="after-abort")


@pytest.mark.parametrize("h, plan", [
    (0.05, None),
    (-0.08, dict(mode=TILED, tile_planes=8, sweeps_per_launch=2, block_threads=256)),
    (0.1, dict(mode=FUSED, block_threads=256)),
    (0.3, dict(mode=TILED, tile_planes=32, sweeps_per_launch=5, block_threads=256)),
])
def test_field(pt, oracle_mod, h, plan):
    """h != 0: ten flip classes and the factorised field swap rule."""
    beta = beta_linear(0.30, 0.55, 6)
    rec = 60
    cfg_kw = dict(seed=19, record_every=1, max_records=rec)
    sim = pt.Simulation(pt.Config(0, 32, 6, beta, h=h, **cfg_kw))
    if plan is not None:
        sim.set_plan(**plan)
    orc = oracle_mod.Oracle(0, 32, 6, beta, h=h, **cfg_kw)
    say("case field h", h, "plan", plan)
    sim.run(rec, 1)
    orc.run(rec, 1)
    compare(sim, orc, "field")
    assert orc.swaps()[1].sum() > 0


def test_primitive_calls_equal_run(pt, oracle_mod):
    """pt_sweep / pt_exchange in intervals give the same result as pt_run."""
    beta = beta_geometric(0.2, 0.6, 8)
    for plan in (None, dict(mode=TILED, tile_planes=4, sweeps_per_launch=2, block_threads=256)):
        run_case(pt, oracle_mod, 0, 32, 8, beta, 11, 40, 4, plan=plan, split=True, tag="split")


def test_uploaded_spins_and_couplings(pt, oracle_mod):
    rng = np.random.default_rng(5)
    L, R = 8, 4
    N = L ** 3
    J = np.where(rng.random((3, N)) < 0.5, -1, 1).astype(np.int8)
    s0 = np.where(rng.random((R, N)) < 0.3, -1, 1).astype(np.int8)
    beta = beta_geometric(0.6, 2.0, R)
    run_case(pt, oracle_mod, 1, L, R, beta, 9, 30, 2, init_spins=s0, couplings=J, tag="upload")
    s2 = np.where(rng.random((3, 32 * 32)) < 0.5, -1, 1).astype(np.int8)
    run_case(pt, oracle_mod, 0, 32, 3, beta_linear(0.3, 0.6, 3), 2, 30, 2, init_spins=s2,
             plan=dict(mode=TILED, tile_planes=8, sweeps_per_launch=1, block_threads=256),
             tag="upload2d")


def test_beta_zero_negates_every_sweep(pt, oracle_mod):
    """At beta = 0 every attempt flips: after t sweeps each state is (-1)^t times its start."""
    from paper_2512_03825_amd import pt as ptm
    L, R = 32, 4
    sim = make_gpu(ptm, 0, L, R, np.zeros(R), 3, record_every=1, max_records=16,
                   plan=dict(mode=TILED, tile_planes=8, sweeps_per_launch=2, block_threads=256))
    s0 = sim.observables(spins="all")["spins"].copy()
    sim.run(5, 1)
    obs = sim.observables(spins="all")
    wat = obs["walker_at"]
    np.testing.assert_array_equal(obs["spins"], -s0[wat])


@pytest.mark.parametrize("L, R, every, h, split", [
    (8, 5, 3, 0.0, False),
    (16, 70, 10, 0.0, False),     # two waves of walkers, the second partly empty
    (16, 9, 1, 0.15, True),       # field swaps, primitive calls
    (8, 1, 0, 0.0, False),        # one walker, no exchange
])
def test_lanes_plan_matches_oracle(pt, oracle_mod, L, R, every, h, split):
    """The replica-per-lane plan (the paper's decomposition) against the oracle."""
    beta = beta_linear(0.25, 0.7, R)
    sweeps = 60
    tag = "lanes L%d R%d" % (L, R)
    say("case", tag, "every", every, "h", h)
    cfg = pt.Config(0, L, R, beta, h=h, seed=21, stream_id=3, record_every=1, max_records=sweeps)
    sim = pt.Simulation(cfg)
    sim.set_plan(LANES)
    assert sim.plan()["mode"] == LANES
    orc = oracle_mod.Oracle(0, L, R, beta, h=h, seed=21, stream_id=3, record_every=1,
                            max_records=sweeps)
    if split:
        for _ in range(sweeps // every):
            sim.sweep(every)
            sim.exchange()
            orc.sweep(every)
            orc.exchange()
    else:
        sim.run(sweeps, every)
        orc.run(sweeps, every)
    compare(sim, orc, tag)


@pytest.mark.parametrize("L, R, every, h, split, rec", [
    (8, 5, 3, 0.0, False, 1),
    (16, 32, 10, 0.0, False, 1),     # the largest R at L = 16: 1024 lanes
    (16, 9, 1, 0.15, True, 1),       # field swaps, primitive calls
    (8, 1, 0, 0.0, False, 1),        # one walker, no exchange
    (8, 128, 2, 0.05, False, 3),     # the largest R at L = 8, records every third sweep
    (16, 3, 7, -0.1, False, 0),      # no records, odd R
    (16, 2, 1, 0.0, False, 2),       # two walkers in one wavefront
    (16, 1, 1, 0.0, True, 1),        # one walker, exchange steps with no pair
])
def test_wave_plan_matches_oracle(pt, oracle_mod, L, R, every, h, split, rec):
    """Walkers held in the registers of one wavefront's lanes, against the oracle."""
    beta = beta_linear(0.25, 0.7, R)
    sweeps = 60
    tag = "wave L%d R%d" % (L, R)
    say("case", tag, "every", every, "h", h, "rec", rec)
    nrec = sweeps // rec if rec else 0
    cfg = pt.Config(0, L, R, beta, h=h, seed=23, stream_id=4, record_every=rec, max_records=nrec)
    sim = pt.Simulation(cfg)
    sim.set_plan(WAVE)
    assert sim.plan()["mode"] == WAVE
    assert sim.plan()["block_threads"] == (R * L * L // 8 + 63) // 64 * 64
    orc = oracle_mod.Oracle(0, L, R, beta, h=h, seed=23, stream_id=4, record_every=rec,
                            max_records=nrec)
    if split:
        for _ in range(sweeps // every):
            sim.sweep(every)
            sim.exchange()
            orc.sweep(every)
            orc.exchange()
    else:
        sim.run(sweeps, every)
        orc.run(sweeps, every)
    compare(sim, orc, tag)


def test_wave_plan_rejects_other_shapes(pt):
    for model, L, R in ((0, 32, 4), (1, 8, 4), (0, 16, 33), (0, 8, 129)):
        beta = beta_linear(0.3, 0.5, R)
        sim = pt.Simulation(pt.Config(model, L, R, beta, seed=1))
        with pytest.raises(pt.PTError):
            sim.set_plan(WAVE)
        sim.close()


def test_lanes_plan_rejects_other_shapes(pt):
    for model, L, R in ((0, 32, 4), (1, 8, 4), (0, 16, 1100)):
        beta = beta_linear(0.3, 0.5, R)
        sim = pt.Simulation(pt.Config(model, L, R, beta, seed=1))
        with pytest.raises(pt.PTError):
            sim.set_plan(LANES)
        sim.close()


@pytest.mark.parametrize("model, L, R, sweeps, every", [
    (0, 2048, 3, 4, 2),    # automatic plan: 128-row tiles
    (0, 4096, 2, 2, 1),    # 64-row tiles, exchange after every sweep
    (1, 64, 3, 3, 1),      # largest EA lattice, tiled 3D plan
])
def test_large_lattices_match_oracle(pt, oracle_mod, model, L, R, sweeps, every):
    """Larger sides than the benchmark's, through their automatic plans."""
    beta = beta_geometric(0.5, 3.0, R) if model == 1 else beta_linear(0.35, 0.50, R)
    run_case(pt, oracle_mod, model, L, R, beta, 17, sweeps, every, coupling_seed=9,
             tag="large L%d" % L)


def test_largest_2d_lattice_bookkeeping(pt):
    """2D L = 16384 (the largest side): after a few sweeps and exchanges the
    incrementally tracked E and M of every slot equal a recount from the
    returned spins, and the walker map is a permutation."""
    L, R = 16384, 2
    beta = beta_linear(0.40, 0.45, R)
    say("case largest 2D L", L, "R", R)
    sim = make_gpu(pt, 0, L, R, beta, 23, record_every=0, max_records=0)
    sim.run(3, 1)
    obs = sim.observables(spins="all", series=False)
    assert sorted(obs["walker_at"].tolist()) == list(range(R))
    for k in range(R):
        s = obs["spins"][k].reshape(L, L).astype(np.int32)
        E = -int((s * np.roll(s, 1, axis=0)).sum() + (s * np.roll(s, 1, axis=1)).sum())
        assert obs["E_slot"][k] == E, k
        assert obs["M_slot"][k] == int(s.sum()), k
    assert obs["sweeps_done"] == 3 and obs["exchanges_done"] == 3
    sim.close()
