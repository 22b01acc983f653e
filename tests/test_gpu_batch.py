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
