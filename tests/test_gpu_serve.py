"""Served form: jobs of mixed model, size and schedule submitted at different
times to a server whose arena holds only a few of them at once.  Each job's
results must be bit-identical to the same job run alone (the plain path, and
for the small ones the oracle), whatever else was resident while it ran."""
import time

import numpy as np
import pytest

from gpu_common import requires_gpu, say
from paper_2512_03825_amd.workloads import beta_geometric, beta_linear

pytestmark = [pytest.mark.gpu, requires_gpu]

# (model, L, R, sweeps, exchange_every, record_every, h, keep_spins)
JOBS = [
    (0, 16, 8, 60, 10, 1, 0.0, True),
    (0, 32, 16, 45, 5, 3, 0.07, False),
    (0, 64, 12, 33, 0, 0, 0.0, True),
    (0, 128, 20, 50, 10, 2, -0.05, False),
    (0, 256, 5, 25, 5, 1, 0.0, True),
    (0, 512, 4, 24, 4, 2, 0.0, True),     # batched lane, one walker per workgroup
    (0, 1024, 3, 20, 10, 1, 0.0, False),  # tiled lane
    (0, 1024, 5, 17, 5, 1, 0.0, True),    # tiled lane, batched with the one above
    (0, 2048, 2, 12, 3, 2, 0.0, True),    # tiled lane, 64-row tiles
    (1, 8, 24, 70, 1, 1, 0.0, True),
    (1, 16, 10, 40, 3, 1, 0.0, False),
    (1, 32, 6, 30, 10, 5, 0.0, True),
    (0, 16, 64, 200, 10, 10, 0.0, False),
    (0, 64, 33, 35, 7, 1, 0.02, False),
]


def _cfg(pt, i, spec):
    model, L, R, sweeps, every, rec, h, _ = spec
    beta = beta_geometric(0.5, 3.0, R) if model == 1 else beta_linear(0.30, 0.55, R)
    return pt.Config(model, L, R, beta, h=h, seed=5, stream_id=1000 + i, coupling_seed=50 + i,
                     record_every=rec, max_records=(sweeps // rec) if rec else 0)


def _alone(pt, cfg, sweeps, every):
    sim = pt.Simulation(cfg)
    sim.run(sweeps, every)
    obs = sim.observables(spins="all")
    sim.close()
    return obs


def _same(a, b, tag, spins):
    keys = ["E_slot", "M_slot", "walker_at", "swap_att", "swap_acc", "E_series", "M_series"]
    for k in keys:
        np.testing.assert_array_equal(a[k], b[k], err_msg="%s %s" % (tag, k))
    for k in ("sweeps_done", "exchanges_done", "n_records"):
        assert a[k] == b[k], (tag, k)
    if spins:
        np.testing.assert_array_equal(a["spins"], b["spins"], err_msg=tag + " spins")


def _run_to_completion(srv, n, limit_s=120.0):
    t0 = time.time()
    finished = []
    while len(finished) < n:
        srv.step(wait_us=2000)
        finished += srv.done()
        assert time.time() - t0 < limit_s, "served jobs did not finish in time"
    return finished


@pytest.mark.parametrize("arena_scale, classes", [(1.3, (4096, 65536)), (8.0, (4096, 65536)), (8.0, ()),
                                                   (8.0, (300,)), (8.0, (256, 4096, 65536))])
def test_jobs_in_the_mix_equal_jobs_alone(oracle_mod, arena_scale, classes):
    from paper_2512_03825_amd import pt
    cfgs = [_cfg(pt, i, s) for i, s in enumerate(JOBS)]
    biggest = max(pt.pt_workspace_bytes(c) for c in cfgs)
    arena = int(biggest * arena_scale)
    say("served: %d jobs, arena %d bytes (largest job %d)" % (len(JOBS), arena, biggest))
    srv = pt.Server(arena, max_jobs=8, max_walkers=96, tiled_lanes=2, depth=2, cycle_sweeps=4,
                    tiled_sweeps=6, class_sites=classes)
    ids = {}
    # arrivals in three waves, the later ones while earlier jobs are on the device
    for wave in (range(0, 4), range(4, 8), range(8, len(JOBS))):
        for i in wave:
            ids[srv.submit(cfgs[i], JOBS[i][3], JOBS[i][4], keep_spins=JOBS[i][7])] = i
        for _ in range(3):
            srv.step(wait_us=500)
    finished = _run_to_completion(srv, len(JOBS))
    st = srv.stats()
    say("served stats", st)
    assert st["finished"] == len(JOBS) and st["resident"] == 0 and st["pending"] == 0
    assert st["arena_used"] == 0 and st["arena_peak"] <= st["arena_bytes"]
    assert {f["job_id"] for f in finished} == set(ids)
    for f in finished:
        assert f["arrival"] <= f["admitted"] <= f["finished"]
        i = ids[f["job_id"]]
        # replicas up to 2D 512^2 (4 bits per site) and EA 32^3 fit one workgroup's LDS;
        # the others take the batched lane of the first size class that holds them
        # (lanes 3, 4, ... after the two tiled lanes), lane 0 if none does
        model, L = JOBS[i][0], JOBS[i][1]
        sites = L ** (3 if model else 2)
        if model == 0 and L >= 1024:
            want = (1, 2)
        else:
            want = (next((3 + k for k, b in enumerate(classes) if sites <= b), 0),)
        assert f["lane"] in want, (i, f["lane"], want)
    for jid, i in ids.items():
        model, L, R, sweeps, every, rec, h, keep = JOBS[i]
        say("job", i, "model", model, "L", L, "R", R)
        got = srv.result(jid, spins="all" if keep else None)
        want = _alone(pt, cfgs[i], sweeps, every)
        _same(got, want, "job %d" % i, keep)
        srv.release(jid)
    srv.close()


def test_small_served_jobs_equal_the_oracle(oracle_mod):
    from paper_2512_03825_amd import pt
    picks = [0, 7]  # 2D 16^2 and EA 8^3
    cfgs = {i: _cfg(pt, i, JOBS[i]) for i in picks}
    srv = pt.Server(4 << 20, max_jobs=4, max_walkers=64)
    ids = {srv.submit(cfgs[i], JOBS[i][3], JOBS[i][4], keep_spins=True): i for i in picks}
    _run_to_completion(srv, len(picks))
    for jid, i in ids.items():
        model, L, R, sweeps, every, rec, h, _ = JOBS[i]
        beta = beta_geometric(0.5, 3.0, R) if model == 1 else beta_linear(0.30, 0.55, R)
        o = oracle_mod.Oracle(model, L, R, beta, h=h, seed=5, stream_id=1000 + i,
                              coupling_seed=50 + i, record_every=rec, max_records=sweeps // rec)
        o.run(sweeps, every)
        got = srv.result(jid, spins="all")
        Es, Ms = o.series()
        np.testing.assert_array_equal(got["E_series"], Es)
        np.testing.assert_array_equal(got["M_series"], Ms)
        E, M = o.energy()
        np.testing.assert_array_equal(got["E_slot"], E)
        np.testing.assert_array_equal(got["M_slot"], M)
        np.testing.assert_array_equal(got["walker_at"], o.labels())
        np.testing.assert_array_equal(got["spins"], o.spins())
        att, acc = o.swaps()
        for k in range(R - 1):
            assert got["swap_att"][k, k + 1] == att[k] and got["swap_acc"][k, k + 1] == acc[k]
    srv.close()


def test_server_rejects_invalid_jobs():
    from paper_2512_03825_amd import pt
    srv = pt.Server(1 << 20, max_jobs=2, max_walkers=16)
    good = pt.Config(0, 16, 4, beta_linear(0.3, 0.5, 4), seed=1)
    with pytest.raises(pt.PTError):
        srv.submit(good, 0, 10)  # no sweeps
    with pytest.raises(pt.PTError):
        srv.submit(pt.Config(0, 16, 4, beta_linear(0.3, 0.5, 4), record_every=1, max_records=5), 10, 5)
    with pytest.raises(pt.PTError):
        srv.submit(pt.Config(0, 16, 4, beta_linear(0.3, 0.5, 4),
                             init_spins=np.ones((4, 256), np.int8)), 10, 5)
    with pytest.raises(pt.PTError):
        srv.submit(pt.Config(0, 1024, 64, beta_linear(0.3, 0.5, 64)), 10, 5)  # larger than the arena
    with pytest.raises(pt.PTError):
        srv.submit(pt.Config(0, 16, 32, beta_linear(0.3, 0.5, 32)), 10, 5)  # more walkers than allowed
    jid = srv.submit(good, 10, 5)
    with pytest.raises(pt.PTError):
        srv.result(jid)  # not finished yet
    _run_to_completion(srv, 1)
    assert srv.result(jid)["sweeps_done"] == 10
    srv.release(jid)
    srv.close()


def test_tiled_lane_job_equals_the_oracle(oracle_mod):
    """A 1024^2 job runs on a tiled lane (its replicas do not fit one
    workgroup's LDS), next to a batched job; its results, final spins included,
    equal the oracle's."""
    from paper_2512_03825_amd import pt
    L, R, sweeps, every = 1024, 4, 20, 5
    beta = beta_linear(0.4400, 0.4401, R)   # narrow: swaps are accepted
    big = pt.Config(0, L, R, beta, seed=5, stream_id=2024, record_every=1, max_records=sweeps)
    small = _cfg(pt, 0, JOBS[0])
    srv = pt.Server(64 << 20, max_jobs=4, max_walkers=64, tiled_lanes=1, tiled_sweeps=4)
    jid = srv.submit(big, sweeps, every, keep_spins=True)
    srv.submit(small, JOBS[0][3], JOBS[0][4])
    finished = _run_to_completion(srv, 2)
    lane = {f["job_id"]: f["lane"] for f in finished}[jid]
    assert lane == 1, lane   # the tiled lane
    o = oracle_mod.Oracle(0, L, R, beta, seed=5, stream_id=2024, record_every=1, max_records=sweeps)
    o.run(sweeps, every)
    got = srv.result(jid, spins="all")
    Es, Ms = o.series()
    np.testing.assert_array_equal(got["E_series"], Es)
    np.testing.assert_array_equal(got["M_series"], Ms)
    np.testing.assert_array_equal(got["walker_at"], o.labels())
    att, acc = o.swaps()
    for k in range(R - 1):
        assert got["swap_att"][k, k + 1] == att[k] and got["swap_acc"][k, k + 1] == acc[k]
    assert sum(acc) > 0
    np.testing.assert_array_equal(got["spins"], o.spins())
    srv.close()
