"""Write the stored expected values of the full-size parity tests.

Calls only the CPU oracle.  For each case it runs a prefix of a full-size
schedule (the oracle needs about a minute per 2*10^9 flip attempts) and stores
the E/M record series, the walker map, the swap counts and a SHA-256 of the
final spins of every slot (+-1 bytes in slot order, each slot's sites in site
order).

Cases:
  ising2d_L1024_R64          the 1024^2 x 64 workload as specified (beta linear
                             0.30..0.55), 100 sweeps, an exchange step every 10
                             (10 steps; the ladder is wide, so none is accepted)
  ising2d_L1024_R64_narrow   the same lattice, seed and replica count on a ladder
                             narrow enough that swaps are accepted (beta linear
                             0.4400..0.4401, exchange every 5, 100 sweeps, 20
                             steps), so that the slot changes of the benchmarked
                             launch configuration are compared at full size
  ea3d_L32_R128              the EA 32^3 x 128 workload, 60 sweeps, an exchange
                             step after every sweep

    python tests/golden/make_golden.py            # all cases
    python tests/golden/make_golden.py ea3d_L32_R128
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2512_03825_amd.workloads import HOT_PATH, beta_linear  # noqa: E402


def _case(base, sweeps, beta=None, exchange_every=None, require_accepts=False):
    return dict(base=base, sweeps=sweeps, beta=beta, exchange_every=exchange_every,
                require_accepts=require_accepts)


CASES = {
    "ising2d_L1024_R64": _case("ising2d_L1024_R64", 100),
    "ising2d_L1024_R64_narrow": _case("ising2d_L1024_R64", 100, beta=beta_linear(0.4400, 0.4401, 64),
                                      exchange_every=5, require_accepts=True),
    "ea3d_L32_R128": _case("ea3d_L32_R128", 60),
}


def make(name):
    c = CASES[name]
    w = HOT_PATH[c["base"]]
    beta = w.beta if c["beta"] is None else np.asarray(c["beta"], np.float64)
    every = w.exchange_every if c["exchange_every"] is None else c["exchange_every"]
    n = c["sweeps"]
    t0 = time.time()
    o = oracle.Oracle(w.model, w.L, w.R, beta, J=w.J, seed=w.seed, coupling_seed=w.coupling_seed,
                      record_every=w.record_every, max_records=n)
    o.run(n, every)
    E, M = o.series()
    att, acc = o.swaps()
    if c["require_accepts"] and int(np.sum(acc)) == 0:
        raise SystemExit("%s: no swap was accepted; the case would not exercise slot changes" % name)
    spins = o.spins()
    out = {
        "workload": c["base"], "case": name, "sweeps": n, "exchange_every": every,
        "record_every": w.record_every, "seed": w.seed, "coupling_seed": w.coupling_seed,
        "L": w.L, "R": w.R, "model": w.model,
        "beta": [float(b) for b in beta],
        "E_series": E.tolist(), "M_series": M.tolist(),
        "labels": o.labels().tolist(), "swap_att": att.tolist(), "swap_acc": acc.tolist(),
        "spins_sha256": hashlib.sha256(spins.tobytes()).hexdigest(),
        "note": "written by tests/golden/make_golden.py from the CPU oracle",
    }
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("%s: %d sweeps in %.1f s, %d swaps accepted -> %s"
          % (name, n, time.time() - t0, int(np.sum(acc)), path), flush=True)


if __name__ == "__main__":
    oracle.build(force=False)
    for name in (sys.argv[1:] or list(CASES)):
        make(name)
