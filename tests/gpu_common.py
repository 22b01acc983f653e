"""Helpers shared by the GPU parity tests: run one configuration on the GPU
library and on the CPU oracle and compare every output element by element."""
import sys

import numpy as np
import pytest


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


requires_gpu = pytest.mark.skipif(not gpu_available(), reason="no GPU visible")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_gpu(pt, model, L, R, beta, seed, coupling_seed=None, init_spins=None, couplings=None,
             record_every=1, max_records=0, plan=None, J=1.0, stream_id=0):
    cfg = pt.Config(model, L, R, beta, J=J, seed=seed, stream_id=stream_id,
                    coupling_seed=coupling_seed, init_spins=init_spins, couplings=couplings,
                    record_every=record_every, max_records=max_records)
    sim = pt.Simulation(cfg)
    if plan is not None:
        sim.set_plan(**plan)
    return sim


def make_oracle(oracle, model, L, R, beta, seed, coupling_seed=None, init_spins=None,
                couplings=None, record_every=1, max_records=0, J=1.0, stream_id=0):
    return oracle.Oracle(model, L, R, beta, J=J, seed=seed, stream_id=stream_id,
                         coupling_seed=coupling_seed, init_spins=init_spins, couplings=couplings,
                         record_every=record_every, max_records=max_records)


def compare(sim, orc, tag=""):
    """Bit-exact comparison of every observable of a GPU simulation and the oracle."""
    obs = sim.observables(spins="all")
    R = orc.R
    np.testing.assert_array_equal(obs["walker_at"], orc.labels(), err_msg=tag + " walker_at")
    Es, Ms = orc.series()
    assert obs["n_records"] == orc.n_records, tag
    np.testing.assert_array_equal(obs["E_series"], Es, err_msg=tag + " E series")
    np.testing.assert_array_equal(obs["M_series"], Ms, err_msg=tag + " M series")
    E, M = orc.energy()
    np.testing.assert_array_equal(obs["E_slot"], E, err_msg=tag + " E")
    np.testing.assert_array_equal(obs["M_slot"], M, err_msg=tag + " M")
    att, acc = orc.swaps()
    for k in range(R - 1):
        assert obs["swap_att"][k, k + 1] == att[k] == obs["swap_att"][k + 1, k], (tag, k)
        assert obs["swap_acc"][k, k + 1] == acc[k] == obs["swap_acc"][k + 1, k], (tag, k)
    assert obs["sweeps_done"] == orc.sweeps_done and obs["exchanges_done"] == orc.exchanges_done
    sp = orc.spins()
    if not np.array_equal(obs["spins"], sp):
        bad = np.argwhere(obs["spins"] != sp)
        raise AssertionError("%s spins differ at %d sites, first %s" % (tag, len(bad), bad[:5].tolist()))
    return obs
