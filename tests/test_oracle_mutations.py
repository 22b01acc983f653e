"""The oracle's pins have teeth: plant a plausible mistake in a copy of
oracle.c (on the CPU), rebuild it, and check that the pin meant to catch that
kind of mistake fails.  The real oracle is never modified."""
import os
import shutil
import tempfile

import pytest

import test_oracle_pins as pins

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle", "oracle.c")

# (name, text in oracle.c, planted replacement, pin expected to fail)
MUTATIONS = [
    ("swap sign", "double x = (beta_k - beta_k1) * dE;", "double x = (beta_k1 - beta_k) * dE;",
     pins.test_swaps_preserve_each_slot_distribution),
    ("half beta in Eq. 1", "exp(-(beta * dE))", "exp(-(0.5 * beta * dE))",
     pins.test_brute_force_ising_4x4),
    ("bond owner of the -d neighbour", "int64_t owner = (dir > 0) ? i : neighbour(st, i, d, -1);",
     "int64_t owner = i;", pins.test_ea_gauge_invariance),
    ("Weyl key constant", "k0 += 0x9E3779B9u;", "k0 += 0x9E3779BBu;",
     pins.test_philox_matches_aten),
    ("dropped factor 2 in dE_int", "st->E[k] += 2 * si * F;", "st->E[k] += si * F;",
     pins.test_incremental_energy_equals_recount),
    ("first pairing shifted", "for (int k = (int)(e & 1u); k + 1 < R; k += 2) {",
     "for (int k = (int)((e + 1u) & 1u); k + 1 < R; k += 2) {",
     pins.test_exchange_schedule_alternates_pairs),
    ("field sign in the swap factor", "double y = (dbeta * -cfg->h) * (double)dM;",
     "double y = (dbeta * cfg->h) * (double)dM;",
     lambda m: pins.test_field_swaps_preserve_each_slot_distribution(m, 0.3)),
    ("flip sign of the spin in dE", "(2.0 * (double)si) * (cfg->J * (double)F + cfg->h)",
     "(-2.0 * (double)si) * (cfg->J * (double)F + cfg->h)", pins.test_ordered_state_is_ground_state),
]


@pytest.mark.parametrize("name, old, new, pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, pin):
    import oracle
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, name
    with tempfile.TemporaryDirectory() as d:
        shutil.copy(os.path.join(os.path.dirname(ORACLE_SRC), "oracle.h"), d)
        path = os.path.join(d, "oracle_mutant.c")
        open(path, "w").write(src.replace(old, new))
        lib = oracle.compile_source(path, os.path.join(d, "libmutant.so"))
        mutant = oracle.bind(lib)
        with pytest.raises(AssertionError):
            pin(mutant)
