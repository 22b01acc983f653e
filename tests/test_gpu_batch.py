"""Batched form: instances of mixed size and model advanced together
(online-tuned decompositions, graph-replayed cycles) are each bit-identical to
the oracle run alone with the same configuration."""
import numpy as np
import pytest

from gpu_common import compare, requires_gpu, say
from paper_2512_03825_amd.workloads import beta_geometric, beta_linear

pytestmark = [pytest.mark.gpu, requires_gpu]


class _Obs:
    """Adapter so gpu_common.compare can read a batch instance."""

    def __init__(self, batch, i):
        self.batch, self.i = batch, i

    def observables(self, spins=None):
        return self.batch.observables(self.i, spins=spins)


def _instances(rng, n):
    out = []
    for i in range(n):
        if i % 4 == 3:
            L, R, model = int(rng.choice([8, 16])), int(rng.integers(2, 7)), 1
            beta, h = beta_geometric(0.5, 2.5, R), 0.0
        else:
            L, R, model = int(rng.choice([8, 16, 32, 64])), int(rng.integers(2, 9)), 0
            beta, h = beta_linear(0.30, 0.55, R), float(rng.uniform(-0.1, 0.1))
        out.append(dict(model=model, L=L, R=R, beta=beta, h=h, seed=4, stream_id=i,
                        coupling_seed=4 + i))
    return out


@pytest.mark.parametrize("every, sweeps", [(5, 60), (1, 23), (0, 37)])
def test_batch_matches_oracle_per_instance(oracle_mod, every, sweeps):
    from paper_2512_03825_amd import pt
    rng = np.random.default_rng(every * 100 + sweeps)
    specs = _instances(rng, 12)
    cfgs = [pt.Config(s["model"], s["L"], s["R"], s["beta"], h=s["h"], seed=s["seed"],
                      stream_id=s["stream_id"], coupling_seed=s["coupling_seed"], record_every=1,
                      max_records=sweeps) for s in specs]
    say("batch", len(cfgs), "instances, every", every, "sweeps", sweeps)
    batch = pt.Batch(cfgs)
    # two runs: the first includes the online tuning cycles, the second replays the graph
    first = sweeps // 3
    batch.run(first, every)
    batch.run(sweeps - first, every)
    say("group plans", batch.group_plans())
    for i, s in enumerate(specs):
        orc = oracle_mod.Oracle(s["model"], s["L"], s["R"], s["beta"], h=s["h"], seed=s["seed"],
                                stream_id=s["stream_id"], coupling_seed=s["coupling_seed"],
                                record_every=1, max_records=sweeps)
        orc.run(first, every)
        orc.run(sweeps - first, every)
        compare(_Obs(batch, i), orc, "batch instance %d %s" % (i, {k: s[k] for k in ("model", "L", "R")}))
    batch.close()


def test_batched2048_shapes_match_oracle(oracle_mod):
    """Instances of the 2048-instance workload itself (seed 4, their own stream
    ids, fields and ladders): for every lattice size L in {32, 64, 128, 256} and
    replica count R in {16, 32, 64} the first such instance of the workload, 12
    in all, advanced together with an exchange step every 5 sweeps.  The first
    run covers the online tuning cycles (every candidate decomposition of every
    group, including one walker per workgroup for L = 128 and 256), the second
    the graph replay of the chosen ones; each instance is compared with the
    oracle run alone."""
    from paper_2512_03825_amd import pt
    from paper_2512_03825_amd.workloads import batched2048
    ws = batched2048()
    picks = {}
    for w in ws:
        picks.setdefault((w.L, w.R), w)
    assert len(picks) == 12 and all(w.h != 0.0 for w in picks.values())
    specs = [picks[k] for k in sorted(picks)]
    first, second = 60, 20
    sweeps = first + second
    cfgs = [pt.Config(w.model, w.L, w.R, w.beta, h=w.h, seed=w.seed, stream_id=w.stream_id,
                      record_every=1, max_records=sweeps) for w in specs]
    say("batched2048 shapes:", [(w.name, w.L, w.R, round(w.h, 4)) for w in specs])
    batch = pt.Batch(cfgs)
    batch.run(first, specs[0].exchange_every)
    batch.run(second, specs[0].exchange_every)
    plans = batch.group_plans()
    say("group plans", plans)
    for i, w in enumerate(specs):
        say("instance", w.name, "L", w.L, "R", w.R)
        orc = oracle_mod.Oracle(w.model, w.L, w.R, w.beta, h=w.h, seed=w.seed, stream_id=w.stream_id,
                                record_every=1, max_records=sweeps)
        orc.run(first, w.exchange_every)
        orc.run(second, w.exchange_every)
        compare(_Obs(batch, i), orc, "%s L %d R %d" % (w.name, w.L, w.R))
    batch.close()


def _tuning_batch(pt):
    from paper_2512_03825_amd.workloads import beta_linear
    cfgs = []
    for i, (L, R) in enumerate([(32, 4), (64, 8), (64, 3), (128, 4), (32, 6), (128, 2)]):
        cfgs.append(pt.Config(0, L, R, beta_linear(0.30, 0.55, R), h=0.03 * (i - 2), seed=4,
                              stream_id=i, record_every=5, max_records=40))
    return pt.Batch(cfgs), len(cfgs)


def _digest(batch, n):
    import hashlib
    h = hashlib.sha256()
    for i in range(n):
        o = batch.observables(i, spins="all")
        for k in ("spins", "E_series", "M_series", "walker_at", "swap_acc"):
            h.update(np.ascontiguousarray(o[k]).tobytes())
    return h.hexdigest()


def test_tuning_cache_file_decides_the_next_batch(tmp_path, monkeypatch):
    """The online tuner's choices (walkers per workgroup and block size per
    lattice-size group, sweeps per cycle per mix of groups and interval) are
    written to the cache file, and a cache file alone decides a new batch's
    decompositions: pointing PTMI_TUNE_CACHE at a copy of the file (the
    library then drops what it holds and reads the copy, as a new process
    would) gives a batch that starts with the first batch's final
    decompositions, runs the same cycle length without tuning, and ends bit
    for bit where the first one did; a hand-written entry is taken as given."""
    from paper_2512_03825_amd import pt
    first = tmp_path / "first.txt"
    monkeypatch.setenv("PTMI_TUNE_CACHE", str(first))
    b1, n = _tuning_batch(pt)
    b1.run(100, 5)
    after = b1.group_plans()
    d1 = _digest(b1, n)
    b1.close()
    text = first.read_text()
    say("tuning cache:\n" + text)
    assert "group gfx" in text and "cycle gfx" in text and "every=5" in text, text
    for p in after:
        assert ("L=%d" % p["L"]) in text and ("W=%d threads=%d" % (p["walkers_per_wg"], p["block_threads"])) in text
    assert all(p["sweeps_per_cycle"] in (1, 5) for p in after)
    assert ("K=%d" % after[0]["sweeps_per_cycle"]) in text

    copy = tmp_path / "copy.txt"
    copy.write_text(text)
    monkeypatch.setenv("PTMI_TUNE_CACHE", str(copy))
    b2, _ = _tuning_batch(pt)
    strip = lambda plans: [{k: q[k] for k in ("L", "walkers_per_wg", "block_threads")} for q in plans]
    before = b2.group_plans()
    assert strip(before) == strip(after) and all(q["sweeps_per_cycle"] == 0 for q in before)
    b2.run(100, 5)
    assert b2.group_plans() == after
    assert _digest(b2, n) == d1
    b2.close()

    # an entry written by hand (one walker per workgroup of 64 threads for the
    # 64^2 group) is used as given, and changes no result
    hand = tmp_path / "hand.txt"
    hand.write_text("\n".join(l if " L=64 " not in l else l.split(" = ")[0] + " = W=1 threads=64"
                              for l in text.splitlines()) + "\n")
    monkeypatch.setenv("PTMI_TUNE_CACHE", str(hand))
    b3, _ = _tuning_batch(pt)
    p64 = [q for q in b3.group_plans() if q["L"] == 64][0]
    assert (p64["walkers_per_wg"], p64["block_threads"]) == (1, 64)
    b3.run(100, 5)
    assert _digest(b3, n) == d1
    b3.close()
