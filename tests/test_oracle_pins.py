"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

None of these tests compares the oracle with itself: each checks it against an
independent implementation (ATen's Philox engine), an exact enumeration, a
closed form (Onsager, Yang), an exact special case (beta = 0, ordered ground
state) or an exact symmetry of the model (global spin flip, EA gauge).
"""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2512_03825_amd.workloads import beta_geometric, beta_linear

ISING2D, EA3D = 0, 1


# ---------------------------------------------------------------------------
# Philox4x32-10: cross-check against ATen's independent header-only engine.
# at::philox_engine(seed, subsequence, offset) uses key = (seed lo, seed hi),
# counter = (offset lo, offset hi, subsequence lo, subsequence hi) and returns
# the four output words in order on successive calls.
# ---------------------------------------------------------------------------
_ATEN_HARNESS = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cinttypes>
int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    uint64_t seed = ((uint64_t)k1 << 32) | k0;
    uint64_t sub = ((uint64_t)c3 << 32) | c2;
    uint64_t off = ((uint64_t)c1 << 32) | c0;
    at::philox_engine e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


def _aten_philox(rows):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "h.cpp"), os.path.join(d, "h")
        with open(src, "w") as f:
            f.write(_ATEN_HARNESS)
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", inc, src, "-o", exe])
        inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_aten(oracle_mod):
    rng = np.random.default_rng(12345)
    rows = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64).tolist()
    rows += [[0] * 6, [2**32 - 1] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 1 << 8],
             [3, 0, 17, 5, 63, 1], [2, 7, 131071, 9999, 63, 0]]
    ref = _aten_philox(rows)
    for r, want in zip(rows, ref):
        got = oracle_mod.philox4x32_10(r[2:6], r[0:2])
        assert [int(v) for v in got] == [int(v) for v in want], r


def test_philox_output_is_balanced(oracle_mod):
    # 4096 blocks of the flip-draw stream: every output bit is set about half the time.
    words = np.array([oracle_mod.philox4x32_10([j, 7, 3, 0], [1, 0]) for j in range(4096)],
                     dtype=np.uint64).ravel()
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint64)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / math.sqrt(words.size))


# ---------------------------------------------------------------------------
# Acceptance rules (Eq. 1 and the swap probability of Sec. 3).
# ---------------------------------------------------------------------------
def _count_accepts(fn):
    """Number of 32-bit draws r that the (monotone in r) rule accepts."""
    lo, hi = 0, 2**32  # answer in [lo, hi]
    while lo < hi:
        mid = (lo + hi) // 2
        if fn(mid):
            lo = mid + 1
        else:
            hi = mid
    return lo


def test_flip_rule_closed_form(oracle_mod):
    for beta in (0.0, 0.2, 0.4407, 1.0, 3.0):
        for dE in (-8.0, -4.0, 0.0):
            assert _count_accepts(lambda r: oracle_mod.flip_accept(beta, dE, r)) == 2**32
        for dE in (4.0, 8.0, 12.0, 24.0):
            n = _count_accepts(lambda r: oracle_mod.flip_accept(beta, dE, r))
            p = math.exp(-beta * dE)
            assert abs(n / 2**32 - p) <= 2**-32 + 1e-15, (beta, dE)
    # Eq. (1): acceptance depends on beta*dE only
    assert _count_accepts(lambda r: oracle_mod.flip_accept(0.5, 8.0, r)) == \
        _count_accepts(lambda r: oracle_mod.flip_accept(1.0, 4.0, r))


def test_swap_rule_detailed_balance(oracle_mod):
    # Barker form: P(x) + P(-x) = 1 and P(x)/P(-x) = e^x, up to the 2^-32 draw grid.
    for db in (-0.25, -0.004, 0.0, 0.05):
        for dE in (-400.0, -40.0, -4.0, 0.0, 4.0, 40.0, 400.0, 8000.0):
            x = db * dE
            n_plus = _count_accepts(lambda r: oracle_mod.swap_accept(db, 0.0, dE, r))
            n_minus = _count_accepts(lambda r: oracle_mod.swap_accept(db, 0.0, -dE, r))
            assert n_plus + n_minus in (2**32, 2**32 + 1), (db, dE)
            p = 1.0 / (1.0 + math.exp(-x)) if abs(x) < 700 else float(x > 0)
            assert abs(n_plus / 2**32 - p) <= 2 * 2**-32 + 1e-15, (db, dE)
    # swap symmetry: exchanging the labels of the two slots leaves x unchanged
    for r in (0, 1, 2**31, 2**32 - 1, 123456789):
        assert oracle_mod.swap_accept(0.3, 0.5, 12.0, r) == oracle_mod.swap_accept(0.5, 0.3, -12.0, r)


# ---------------------------------------------------------------------------
# Exact enumeration (Eq. 2 and Eq. 3).
# ---------------------------------------------------------------------------
def _enumerate_ising2d(L):
    N = L * L
    states = np.arange(2**N, dtype=np.int64)
    s = (1 - 2 * ((states[:, None] >> np.arange(N)) & 1)).astype(np.int64).reshape(-1, L, L)
    E = -(s * np.roll(s, -1, axis=2)).sum((1, 2)) - (s * np.roll(s, -1, axis=1)).sum((1, 2))
    M = s.sum((1, 2))
    return E, M


def _enumerate_ea3d(L, J):
    N = L**3
    states = np.arange(2**N, dtype=np.int64)
    s = (1 - 2 * ((states[:, None] >> np.arange(N)) & 1)).astype(np.int64).reshape(-1, L, L, L)
    Jz, Jy, Jx = (J[d].reshape(L, L, L).astype(np.int64) for d in (2, 1, 0))  # [z][y][x]
    E = -(Jx * s * np.roll(s, -1, axis=3)).sum((1, 2, 3)) \
        - (Jy * s * np.roll(s, -1, axis=2)).sum((1, 2, 3)) \
        - (Jz * s * np.roll(s, -1, axis=1)).sum((1, 2, 3))
    M = s.reshape(len(states), -1).sum(1)
    return E, M


def _boltzmann_means(E, M, beta):
    w = np.exp(-beta * (E - E.min()))
    Z = w.sum()
    return (E * w).sum() / Z, (np.abs(M) * w).sum() / Z


def _block_stats(x, nblocks):
    x = np.asarray(x, dtype=np.float64)
    n = len(x) // nblocks * nblocks
    b = x[:n].reshape(nblocks, -1).mean(1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nblocks)


def test_brute_force_ising_4x4(oracle_mod):
    """<E> and <|M|> of a 4x4 periodic Ising lattice at the 16x16 ladder's 8 betas."""
    beta = beta_geometric(0.20, 0.60, 8)
    E_all, M_all = _enumerate_ising2d(4)
    n = 200_000
    o = oracle_mod.Oracle(ISING2D, 4, 8, beta, seed=11, record_every=1, max_records=n)
    o.run(n, every=10)
    Es, Ms = o.series()
    burn = 2000
    for k in range(8):
        eE, eM = _boltzmann_means(E_all, M_all, beta[k])
        mE, sE = _block_stats(Es[burn:, k], 100)
        mM, sM = _block_stats(np.abs(Ms[burn:, k]), 100)
        assert abs(mE - eE) < 5 * sE, (k, mE, eE, sE)
        assert abs(mM - eM) < 5 * sM, (k, mM, eM, sM)


def _ea_l2_free_sites(J):
    """Sites of the 2x2x2 torus whose field is identically zero.

    On L = 2 each neighbour pair is joined by two bonds (i -> i+e_d and back);
    when the two have opposite signs along all three axes the site feels no
    field, Metropolis accepts its flip with probability 1 (dE = 0), and a
    checkerboard sweep flips it deterministically every sweep: its phase is
    conserved and the chain is not ergodic.  Such instances are excluded.
    """
    L, N = 2, 8
    i = np.arange(N)
    x, y, z = i % L, (i // L) % L, i // (L * L)
    nb = [((x + 1) % L) + L * y + L * L * z, x + L * ((y + 1) % L) + L * L * z,
          x + L * y + L * L * ((z + 1) % L)]
    return [s for s in range(N) if all(J[d][s] + J[d][nb[d][s]] == 0 for d in range(3))]


@pytest.mark.parametrize("kind", ["random", "ferromagnet"])
def test_brute_force_ea_L2(oracle_mod, kind):
    """3D EA on the 2x2x2 torus (256 states, 24 bonds) at a 6-slot ladder.

    kind='ferromagnet' (all J = +1) is the special case where the EA model
    reduces to the 3D Ising model.
    """
    rng = np.random.default_rng(7)
    if kind == "ferromagnet":
        J = np.ones((3, 8), dtype=np.int8)
    else:
        while True:
            J = np.where(rng.random((3, 8)) < 0.5, -1, 1).astype(np.int8)
            if not _ea_l2_free_sites(J):
                break
    beta = beta_geometric(0.3, 1.5, 6) * (0.5 if kind == "ferromagnet" else 1.0)
    E_all, M_all = _enumerate_ea3d(2, J)
    n = 200_000
    for every in (1, 0):  # with and without replica exchange
        o = oracle_mod.Oracle(EA3D, 2, 6, beta, seed=5, couplings=J, record_every=1,
                              max_records=n)
        o.run(n, every=every)
        Es, Ms = o.series()
        for k in range(6):
            eE, eM = _boltzmann_means(E_all, M_all, beta[k])
            mE, sE = _block_stats(Es[2000:, k], 100)
            mM, sM = _block_stats(np.abs(Ms[2000:, k]), 100)
            assert abs(mE - eE) < 5 * sE, (every, k, mE, eE, sE)
            assert abs(mM - eM) < 5 * sM, (every, k, mM, eM, sM)


def test_swaps_preserve_each_slot_distribution(oracle_mod):
    """Exchange every sweep between 3 slots: each slot still samples its own Boltzmann law."""
    beta = np.array([0.25, 0.40, 0.55])
    E_all, M_all = _enumerate_ising2d(4)
    n = 200_000
    o = oracle_mod.Oracle(ISING2D, 4, 3, beta, seed=21, record_every=1, max_records=n)
    o.run(n, every=1)
    att, acc = o.swaps()
    assert np.all(att > 0) and np.all(acc > 0.05 * att)
    Es, _ = o.series()
    for k in range(3):
        w = np.exp(-beta[k] * (E_all - E_all.min()))
        levels = np.unique(E_all)
        p_exact = np.array([w[E_all == e].sum() for e in levels]) / w.sum()
        mE, sE = _block_stats(Es[1000:, k], 100)
        assert abs(mE - (levels * p_exact).sum()) < 5 * sE
        # histogram of the two most populated levels within 5 sigma (block errors)
        for lev in levels[np.argsort(p_exact)[-2:]]:
            f, sf = _block_stats((Es[1000:, k] == lev).astype(float), 100)
            assert abs(f - p_exact[levels == lev][0]) < 5 * sf + 1e-3


@pytest.mark.parametrize("h", [0.3, -0.2])
def test_field_swaps_preserve_each_slot_distribution(oracle_mod, h):
    """With a field, flips (Eq. 1 with E = -J sum ss - h sum s) and the factorised
    swap rule keep every slot on its exact Boltzmann law: <E_int>, <M>, <|M|>."""
    beta = np.array([0.25, 0.40, 0.55])
    E_all, M_all = _enumerate_ising2d(4)
    n = 200_000
    o = oracle_mod.Oracle(ISING2D, 4, 3, beta, h=h, seed=23, record_every=1, max_records=n)
    o.run(n, every=1)
    att, acc = o.swaps()
    assert np.all(acc > 0.05 * att)
    Es, Ms = o.series()
    for k in range(3):
        logw = -beta[k] * (E_all - h * M_all)
        wts = np.exp(logw - logw.max())
        Z = wts.sum()
        for obs, exact in ((Es[1000:, k], (E_all * wts).sum() / Z),
                           (Ms[1000:, k], (M_all * wts).sum() / Z),
                           (np.abs(Ms[1000:, k]), (np.abs(M_all) * wts).sum() / Z)):
            m, se = _block_stats(obs, 100)
            assert abs(m - exact) < 5 * se, (k, m, exact, se)


# ---------------------------------------------------------------------------
# Closed forms for the infinite 2D Ising model (Onsager 1944, Yang 1952).
# ---------------------------------------------------------------------------
def onsager_energy_per_site(beta):
    from scipy.special import ellipk
    k = 2.0 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2
    K = ellipk(k * k)  # scipy's parameter is m = k^2
    return -1.0 / math.tanh(2 * beta) * (1 + 2 / math.pi * (2 * math.tanh(2 * beta) ** 2 - 1) * K)


def yang_magnetisation(beta):
    return (1.0 - math.sinh(2 * beta) ** -4) ** 0.125


def test_onsager_and_yang(oracle_mod):
    beta = np.array([0.30, 0.34, 0.50, 0.55])
    L, n = 32, 6000
    o = oracle_mod.Oracle(ISING2D, L, 4, beta, seed=31, record_every=1, max_records=n)
    o.run(n, every=10)
    Es, Ms = o.series()
    N = L * L
    for k in (0, 3):
        mE, sE = _block_stats(Es[1000:, k] / N, 50)
        assert abs(mE - onsager_energy_per_site(beta[k])) < 5 * sE + 2e-3, (k, mE)
    mM, sM = _block_stats(np.abs(Ms[1000:, 3]) / N, 50)
    assert abs(mM - yang_magnetisation(0.55)) < 5 * sM + 3e-3, mM
    # disordered side of the transition: |M|/N is small (finite-size scale N^-1/2)
    assert np.abs(Ms[1000:, 0]).mean() / N < 0.15


# ---------------------------------------------------------------------------
# Exact special cases.
# ---------------------------------------------------------------------------
def test_beta_zero_flips_every_site(oracle_mod):
    """At beta = 0 every attempt is accepted, so each sweep negates every state exactly."""
    for model, L in ((ISING2D, 8), (EA3D, 4)):
        R = 4
        o = oracle_mod.Oracle(model, L, R, np.zeros(R), seed=3, record_every=1, max_records=64)
        s0 = o.spins()
        E0, M0 = o.energy()
        for t in range(1, 8):
            o.run(1, every=1)
            lab = o.labels()
            np.testing.assert_array_equal(o.spins(), s0[lab] * (-1) ** t)
            E, M = o.energy()
            np.testing.assert_array_equal(E, E0[lab])
            np.testing.assert_array_equal(M, M0[lab] * (-1) ** t)


def test_ordered_state_is_ground_state(oracle_mod):
    """Start fully aligned at large beta: E stays at the ground-state value -2N."""
    L, R = 16, 4
    beta = np.array([3.0, 3.5, 4.0, 5.0])
    N = L * L
    init = np.ones((R, N), dtype=np.int8)
    init[1] = -1
    o = oracle_mod.Oracle(ISING2D, L, R, beta, seed=9, init_spins=init, record_every=1,
                          max_records=500)
    o.run(500, every=5)
    Es, Ms = o.series()
    assert np.all(Es == -2 * N)
    assert np.all(np.abs(Ms) == N)


def test_global_spin_flip_symmetry(oracle_mod):
    """h = 0: starting from -sigma0 gives the exactly negated trajectory (same E)."""
    L, R = 12, 5
    beta = beta_linear(0.3, 0.55, R)
    probe = oracle_mod.Oracle(ISING2D, L, R, beta, seed=4)
    s0 = probe.spins()
    a = oracle_mod.Oracle(ISING2D, L, R, beta, seed=4, init_spins=s0, record_every=1, max_records=300)
    b = oracle_mod.Oracle(ISING2D, L, R, beta, seed=4, init_spins=-s0, record_every=1, max_records=300)
    a.run(300, every=3)
    b.run(300, every=3)
    np.testing.assert_array_equal(a.spins(), -b.spins())
    np.testing.assert_array_equal(a.labels(), b.labels())
    Ea, Ma = a.series()
    Eb, Mb = b.series()
    np.testing.assert_array_equal(Ea, Eb)
    np.testing.assert_array_equal(Ma, -Mb)
    np.testing.assert_array_equal(a.swaps()[1], b.swaps()[1])


def test_ea_gauge_invariance(oracle_mod):
    """(J_ij, s_i) -> (g_i J_ij g_j, g_i s_i) leaves E and the whole trajectory invariant."""
    L, R = 4, 4
    N = L**3
    beta = beta_geometric(0.5, 2.0, R)
    rng = np.random.default_rng(99)
    J = np.where(rng.random((3, N)) < 0.5, -1, 1).astype(np.int8)
    s0 = np.where(rng.random((R, N)) < 0.5, -1, 1).astype(np.int8)
    g = np.where(rng.random(N) < 0.5, -1, 1).astype(np.int8)
    idx = np.arange(N)
    x, y, z = idx % L, (idx // L) % L, idx // (L * L)
    nb = [((x + 1) % L) + L * y + L * L * z, x + L * ((y + 1) % L) + L * L * z,
          x + L * y + L * L * ((z + 1) % L)]
    Jg = np.stack([J[d] * g * g[nb[d]] for d in range(3)]).astype(np.int8)
    a = oracle_mod.Oracle(EA3D, L, R, beta, seed=8, couplings=J, init_spins=s0,
                          record_every=1, max_records=400)
    b = oracle_mod.Oracle(EA3D, L, R, beta, seed=8, couplings=Jg, init_spins=s0 * g,
                          record_every=1, max_records=400)
    a.run(400, every=1)
    b.run(400, every=1)
    np.testing.assert_array_equal(a.spins() * g, b.spins())
    np.testing.assert_array_equal(a.series()[0], b.series()[0])
    np.testing.assert_array_equal(a.labels(), b.labels())
    assert a.swaps()[1].sum() > 0


def test_incremental_energy_equals_recount(oracle_mod):
    for model, L, R, every in ((ISING2D, 10, 3, 2), (EA3D, 6, 4, 1), (ISING2D, 6, 1, 0)):
        beta = beta_linear(0.1, 1.2, R)
        o = oracle_mod.Oracle(model, L, R, beta, seed=17, J=1.0)
        for _ in range(5):
            o.run(37, every=every)
            E, M = o.energy()
            Er, Mr = o.recount()
            np.testing.assert_array_equal(E, Er)
            np.testing.assert_array_equal(M, Mr)


def test_exchange_schedule_alternates_pairs(oracle_mod):
    """Step 0 pairs (0,1),(2,3),...; step 1 pairs (1,2),(3,4),...; one swap per slot per step."""
    R = 6
    o = oracle_mod.Oracle(ISING2D, 4, R, np.zeros(R), seed=2)
    expected = np.zeros(R - 1, dtype=np.uint64)
    for e in range(5):
        o.exchange()
        expected[e % 2::2] += 1
        att, _ = o.swaps()
        np.testing.assert_array_equal(att, expected)
    # at beta = 0 every pair has x = 0, so it swaps with probability 1/2
    o2 = oracle_mod.Oracle(ISING2D, 4, R, np.zeros(R), seed=2)
    for _ in range(4000):
        o2.exchange()
    att, acc = o2.swaps()
    assert np.all(np.abs(acc / att - 0.5) < 5 * 0.5 / np.sqrt(att))
    assert sorted(o2.labels().tolist()) == list(range(R))


def test_initial_spins_and_couplings_are_fair(oracle_mod):
    o = oracle_mod.Oracle(EA3D, 16, 2, np.ones(2), seed=3, coupling_seed=3)
    s = o.spins().astype(np.int64)
    J = o.couplings().astype(np.int64)
    n = s.size
    assert abs(s.sum()) < 5 * math.sqrt(n)
    assert abs(J.sum()) < 5 * math.sqrt(J.size)
    # distinct slots get distinct initial states
    assert np.mean(s[0] == s[1]) < 0.55


def test_invalid_configs_are_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.Oracle(ISING2D, 5, 2, np.ones(2))
    with pytest.raises(ValueError):
        oracle_mod.Oracle(ISING2D, 4, 2, np.array([1.0, -0.5]))
    with pytest.raises(ValueError):
        oracle_mod.Oracle(ISING2D, 4, 1, np.ones(1), init_spins=np.zeros((1, 16), np.int8))
