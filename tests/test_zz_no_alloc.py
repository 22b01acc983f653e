"""pt_create_static, the entry point that allocates no device memory: its
contexts keep the sweep scratch (per-sweep tallies, exchange mailboxes, split
boundary posts) in the library's fixed per-GPU array.  Every observable must
equal, bit for bit, that of the same configuration created with pt_create, on
two configurations in a row (the second smaller) and when a context resumes
after another one has used the array."""
import numpy as np
import pytest

from gpu_common import requires_gpu, say
from paper_2512_03825_amd.workloads import beta_linear

pytestmark = [pytest.mark.gpu, requires_gpu]


def _pair(pt, model, L, R, beta, seed, sweeps, plan):
    out = []
    for static in (True, False):
        cfg = pt.Config(model, L, R, beta, seed=seed, record_every=1, max_records=sweeps)
        sim = pt.Simulation(cfg, static_scratch=static)
        sim.set_plan(**plan)
        out.append(sim)
    return out


def _same(a, b, tag):
    oa, ob = a.observables(spins="all"), b.observables(spins="all")
    for k in oa:
        if isinstance(oa[k], np.ndarray):
            np.testing.assert_array_equal(oa[k], ob[k], err_msg="%s %s" % (tag, k))
        else:
            assert oa[k] == ob[k], (tag, k)
    return oa


def test_static_scratch_equals_workspace_scratch(pt):
    # call 1: 2D 256^2 x 16 as four row parts per walker (posts and mailboxes),
    # a narrow ladder so that swaps are accepted
    L, R = 256, 16
    beta = beta_linear(0.40, 0.40 + 2.0 / L, R)
    say("static scratch: 2D", L, R, "split P=4")
    big = _pair(pt, 0, L, R, beta, 21, 60, dict(mode=3, tile_planes=64, block_threads=1024))
    state = pt.pt_static_state_bytes(big[0].cfg)
    assert state == big[0].nbytes < pt.pt_workspace_bytes(big[0].cfg)
    for sim in big:
        sim.run(30, 3)
    o = _same(*big, "2D split")
    assert o["swap_acc"].sum() > 0
    # call 2, smaller: EA 16^3 x 8 as two z-plane parts, exchange every sweep
    say("static scratch: EA 16 8 split P=2")
    small = _pair(pt, 1, 16, 8, np.geomspace(0.5, 3.0, 8), 23, 40,
                  dict(mode=3, tile_planes=8, block_threads=512))
    for sim in small:
        sim.run(20, 1)
    _same(*small, "EA split")
    # the first context resumes after the second used the array: tiled plan
    # (per-sweep tallies folded by the last workgroup), then primitive calls
    say("static scratch: 2D resumes, tiled plan and primitive calls")
    for sim in big:
        sim.set_plan(mode=2, tile_planes=64, sweeps_per_launch=2, block_threads=512)
        sim.run(20, 5)
        sim.set_plan(mode=3, tile_planes=64, block_threads=1024)
        sim.sweep(4)
        sim.exchange()
        sim.run(6, 2)
    _same(*big, "2D resumed")
    for sim in small:
        sim.run(20, 1)
    _same(*small, "EA resumed")
    for sim in big + small:
        sim.close()


@pytest.fixture(scope="module")
def pt():
    from paper_2512_03825_amd import pt as _pt
    return _pt
