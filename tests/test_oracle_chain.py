"""Pins for the oracle's Markov chain (Sec. 2.1-2.3) and the weight
iteration as a whole.

  * exact bookkeeping: every histogram sums to walkers * sweeps * N and the
    tracked energy of every walker equals the energy recomputed from its
    lattice;
  * stationarity: with fixed weights omega, independent walkers end in
    states drawn from pi(sigma) ~ exp(omega(E(sigma))), so their energies
    follow g(E) exp(omega(E)) with g from exhaustive enumeration (L = 4)
    or Kaufman's closed form (L = 6);
  * the whole method: after the weight iteration and a production run,
    ln g lies within 0.02 of the exact result (the small workload, L = 4,
    64 walkers, 8 x 2000 sweeps then 20000 production sweeps).
"""
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from muca_inputs import WORKLOADS, random_log_weights
from oracle import exact_dos


def golden_g(golden_dir, L):
    with open(os.path.join(golden_dir, "ising_dos_L%d.txt" % L)) as f:
        return [int(x) for x in f if not x.startswith("#")]


def test_bookkeeping_invariants():
    o = oracle.OracleMuca(6, 37, 5)
    o.set_log_weights(random_log_weights(6, 1, scale=3.0))
    info = o.iterate(3, 11)
    assert info["hist_sum"] == 37 * 36 * 11
    assert int(o.hist.sum()) == 37 * 36 * 11
    assert info["attempts"] == 37 * 36 * 14
    assert o.sweep_counter == 14
    assert o.hist[1] == 0 and o.hist[35] == 0          # forbidden bins
    for w in range(o.W):
        assert o.energies[w] == oracle.energy(6, o.spins[w])
    info = o.production(0, 5)
    assert info["hist_sum"] == 37 * 36 * 5 and o.sweep_counter == 19
    for w in range(o.W):
        assert o.energies[w] == oracle.energy(6, o.spins[w])


def test_first_iteration_is_deterministic():
    # omega = 0: every threshold is 2^32, every proposal is accepted, so one
    # typewriter sweep flips every spin once.
    o = oracle.OracleMuca(8, 5, 3)
    s0 = o.spins.copy()
    o.production(0, 1)
    assert np.array_equal(o.spins, -s0)
    o.production(0, 1)
    assert np.array_equal(o.spins, s0)


def test_split_calls_equal_one_call():
    om = random_log_weights(8, 4, scale=2.0)
    a = oracle.OracleMuca(8, 20, 9)
    a.set_log_weights(om)
    a.production(0, 12)
    b = oracle.OracleMuca(8, 20, 9)
    b.set_log_weights(om)
    hb = b.production(0, 5)["hist_sum"]
    hb += b.production(0, 7)["hist_sum"]
    assert np.array_equal(a.spins, b.spins)
    assert np.array_equal(a.energies, b.energies)
    assert a.sweep_counter == b.sweep_counter == 12
    assert hb == int(a.hist.sum())


def test_attempt_order_is_typewriter():
    # omega = 0 accepts every proposal, so after attempts 0 .. a-1 exactly the
    # sites 0 .. a-1 (p mod N, row by row) are flipped; later calls continue
    # at the next site and wrap into the next sweep.
    L, W = 6, 7
    N = L * L
    o = oracle.OracleMuca(L, W, 4)
    s0 = o.spins.copy()
    flipped = np.zeros(N, dtype=bool)
    for therm, count in [(0, 5), (3, 0), (2, 11), (0, N), (7, 2 * N + 3)]:
        info = o.production_attempts(therm, count)
        for p in range(o.position - therm - count, o.position):
            flipped[p % N] ^= True
        assert info["hist_sum"] == W * count and info["position"] == o.position
        assert np.array_equal(o.spins, np.where(flipped, -s0, s0))
        for w in range(W):
            assert o.energies[w] == oracle.energy(L, o.spins[w])


def test_attempt_split_calls_equal_one_call():
    # any cut of a run into calls, inside sweeps or not, gives the same chain
    L = 8
    N = L * L
    om = random_log_weights(L, 6, scale=2.0)
    a = oracle.OracleMuca(L, 20, 9)
    a.set_log_weights(om)
    a.production_attempts(0, 5 * N + 17)
    b = oracle.OracleMuca(L, 20, 9)
    b.set_log_weights(om)
    total = 0
    for cut in [1, N - 2, 3, 2 * N, 0, N + 5, 5 * N + 17 - (1 + N - 2 + 3 + 2 * N + N + 5)]:
        total += b.production_attempts(0, cut)["hist_sum"]
    assert b.position == a.position == 5 * N + 17
    assert np.array_equal(a.spins, b.spins)
    assert np.array_equal(a.energies, b.energies)
    assert total == int(a.hist.sum())


def test_walker_population_and_threads_do_not_change_results():
    om = random_log_weights(6, 8, scale=2.0)
    runs = []
    for walkers, threads in [(40, 1), (40, 8), (25, 3)]:
        o = oracle.OracleMuca(6, walkers, 21, nthreads=threads)
        o.set_log_weights(om)
        o.production(2, 6)
        runs.append(o)
    assert np.array_equal(runs[0].hist, runs[1].hist)
    assert np.array_equal(runs[0].spins, runs[1].spins)
    assert np.array_equal(runs[0].spins[:25], runs[2].spins)
    assert np.array_equal(runs[0].energies[:25], runs[2].energies)


def test_consecutive_sweeps_use_fresh_random_numbers():
    om = random_log_weights(6, 2, scale=1.0)
    o = oracle.OracleMuca(6, 30, 4)
    o.set_log_weights(om)
    o.production(0, 20)
    h1 = o.hist.copy()
    o.production(0, 20)
    assert not np.array_equal(h1, o.hist)


def _stationary_energy_check(L, g, seed, walkers, sweeps):
    N = L * L
    om = random_log_weights(L, seed, scale=1.5)
    o = oracle.OracleMuca(L, walkers, seed)
    o.set_log_weights(om)
    o.production(20, sweeps)
    reach = oracle.reachable_mask(N)
    logp = np.log(np.array(g, dtype=np.float64)[reach]) + om[reach]
    p = np.exp(logp - logp.max())
    p /= p.sum()
    k = (o.energies.astype(np.int64) + 2 * N) // 4
    counts = np.bincount(k, minlength=N + 1)[reach]
    expected = p * walkers
    # pool sparse bins so that every expected count is at least 5
    order = np.argsort(expected)
    obs_g, exp_g, acc_o, acc_e = [], [], 0.0, 0.0
    for i in order:
        acc_o += counts[i]
        acc_e += expected[i]
        if acc_e >= 5:
            obs_g.append(acc_o)
            exp_g.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0:
        obs_g[-1] += acc_o
        exp_g[-1] += acc_e
    obs_g, exp_g = np.array(obs_g), np.array(exp_g)
    nz = obs_g > 0
    G = 2.0 * np.sum(obs_g[nz] * np.log(obs_g[nz] / exp_g[nz]))
    pval = stats.chi2.sf(G, len(obs_g) - 1)
    # time-averaged histogram of the same run: same law, looser check on
    # the bins that are not rare
    hp = o.hist[reach].astype(np.float64)
    hp /= hp.sum()
    common = p >= 1e-3
    return pval, np.max(np.abs(hp - p)[common] / p[common])


def test_stationary_law_L4_enumeration():
    g = exact_dos.enumerate_dos(4)
    pval, rel = _stationary_energy_check(4, g, seed=11, walkers=40000, sweeps=60)
    assert pval > 1e-6, pval
    assert rel < 0.05, rel


def test_stationary_law_L6_kaufman(golden_dir):
    g = golden_g(golden_dir, 6)
    pval, _ = _stationary_energy_check(6, g, seed=12, walkers=40000, sweeps=80)
    assert pval > 1e-6, pval


def test_stationarity_check_detects_wrong_weights():
    # the same statistic rejects the law with the weights' sign flipped
    g = np.array(exact_dos.enumerate_dos(4), dtype=np.float64)
    om = random_log_weights(4, 11, scale=1.5)
    o = oracle.OracleMuca(4, 40000, 11)
    o.set_log_weights(om)
    o.production(0, 60)
    reach = oracle.reachable_mask(16)
    wrong = np.log(g[reach]) - om[reach]
    p = np.exp(wrong - wrong.max())
    p /= p.sum()
    k = (o.energies.astype(np.int64) + 32) // 4
    counts = np.bincount(k, minlength=17)[reach]
    exp = p * o.W
    keep = exp >= 5
    G = 2.0 * np.sum(np.where(counts[keep] > 0,
                              counts[keep] * np.log(np.maximum(counts[keep], 1) / exp[keep]), 0))
    assert stats.chi2.sf(abs(G), keep.sum() - 1) < 1e-6


def run_workload(name, seed, max_iter=10000):
    wl = WORKLOADS[name]
    o = oracle.OracleMuca(wl["L"], wl["walkers"], seed)
    it = 0
    while True:
        info = o.iterate(wl["therm_sweeps"], wl["iter_sweeps"])
        it += 1
        if wl["iterations"] is not None:
            if it == wl["iterations"]:
                break
        elif info["flatness"] >= wl["min_flat"] or it >= max_iter:
            break
    o.production(wl["prod_therm_sweeps"], wl["prod_sweeps"])
    return o, it


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_small_workload_ln_g_within_0_02(seed):
    o, _ = run_workload("ising_L4_W64", seed)
    lng = o.log_dos(0)
    exact = exact_dos.ln_dos(exact_dos.enumerate_dos(4))
    m = oracle.reachable_mask(16)
    err = np.max(np.abs(lng[m] - exact[m]))
    assert err < 0.02, err
    # the paper's normalisation gives the same curve up to a constant
    lng1 = o.log_dos(1)
    shift = lng1[m] - lng[m]
    assert np.max(shift) - np.min(shift) < 1e-9


def test_L8_converges_to_exact_ln_g(golden_dir):
    L, N = 8, 64
    o = oracle.OracleMuca(L, 512, 3)
    for it in range(200):
        info = o.iterate(0, 100)
        if info["flatness"] >= 0.5:
            break
    assert info["flatness"] >= 0.5
    o.production(0, 4000)
    exact = exact_dos.ln_dos(golden_g(golden_dir, L))
    lng = o.log_dos(0)
    m = oracle.reachable_mask(N)
    err = np.max(np.abs(lng[m] - exact[m]))
    assert err < 0.02, err
