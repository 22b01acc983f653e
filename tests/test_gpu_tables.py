"""The library's FP64-built threshold tables against the oracle's per-decision
rules: for every slot and class, and for swap energy differences inside and
beyond each pair's table window, the number of 32-bit draws the library accepts
equals the number the oracle's rule accepts (exact)."""
import numpy as np
import pytest

from gpu_common import requires_gpu
from paper_2512_03825_amd.workloads import HOT_PATH

pytestmark = [pytest.mark.gpu, requires_gpu]


def n_accepted(rule):
    lo, hi = 0, 2**32
    while lo < hi:
        mid = (lo + hi) // 2
        if rule(mid):
            lo = mid + 1
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("name", list(HOT_PATH))
def test_tables_equal_oracle_rules(oracle_mod, name):
    from paper_2512_03825_amd import pt
    w = HOT_PATH[name]
    L = 8 if w.dim == 3 else 16  # flip tables depend on beta and the model only
    dmax = (2 * w.dim) * L ** w.dim // 4  # |E_a - E_b| / 4 never exceeds this on L^dim sites
    sim = pt.Simulation(pt.Config(w.model, L, w.R, w.beta, J=w.J, seed=w.seed))
    T = pt.pt_flip_thresholds(sim.ctx, w.R)
    z = 2 * w.dim
    for k in range(0, w.R, max(1, w.R // 16)):
        for b in (0, 1):
            for u in range(z + 1):
                s = -1 if b else 1
                F = s * (z - 2 * u)
                dE = (2.0 * s) * (w.J * F + w.h) if w.dim == 2 else (2.0 * s) * F
                want = n_accepted(lambda r: oracle_mod.flip_accept(w.beta[k], dE, r))
                assert int(T[k, 8 * b + u]) + 1 == want, (k, b, u)
    for k in range(0, w.R - 1, max(1, w.R // 8)):
        db = abs(w.beta[k] - w.beta[k + 1])
        D = int(np.ceil((32 * np.log(2) + 1) / (4 * db)))
        for d in sorted({0, 1, -1, 7, -7, D // 3, -D // 3, D - 1, -D + 1, D, -D, D + 1, -D - 1,
                         D + 50, -D - 50, dmax, -dmax}):
            if abs(d) > dmax:
                continue  # unreachable difference: the table is capped there
            got = pt.pt_swap_threshold(sim.ctx, k, d)
            dE = w.J * float(4 * d) if w.dim == 2 else float(4 * d)
            want = n_accepted(lambda r: oracle_mod.swap_accept(w.beta[k], w.beta[k + 1], dE, r))
            assert got == want, (k, d)
    sim.close()
