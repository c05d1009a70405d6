"""Pins for the oracle's model arithmetic: energies, acceptance thresholds,
the weight update, flatness and convergence measures, and ln g.

Energies are pinned by configurations whose energy follows from counting
bonds by hand; thresholds by their closed form at special weight tables
and a value computed at high precision; the host post-processing by
synthetic histograms whose results are known in closed form.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from muca_inputs import random_log_weights
from oracle import exact_dos


# ------------------------------------------------------------------ energies
@pytest.mark.parametrize("L", [4, 6, 8, 32])
def test_energy_special_configurations(L):
    N = L * L
    up = np.ones((L, L), dtype=np.int8)
    assert oracle.energy(L, up) == -2 * N
    assert oracle.energy(L, -up) == -2 * N
    yy, xx = np.mgrid[0:L, 0:L]
    checker = np.where((xx + yy) % 2 == 0, 1, -1).astype(np.int8)
    assert oracle.energy(L, checker) == 2 * N
    one = up.copy()
    one[L // 2, 1] = -1
    assert oracle.energy(L, one) == -2 * N + 8
    stripes = np.where(yy % 2 == 0, 1, -1).astype(np.int8)   # rows alternate
    assert oracle.energy(L, stripes) == 0
    halves = np.where(xx < L // 2, 1, -1).astype(np.int8)     # two vertical walls
    assert oracle.energy(L, halves) == -2 * N + 4 * L
    domino = up.copy()
    domino[0, L - 1] = -1
    domino[0, 0] = -1                                          # across the seam
    assert oracle.energy(L, domino) == -2 * N + 12


def test_init_spins_and_energies():
    o = oracle.OracleMuca(8, 300, 1)
    assert set(np.unique(o.spins).tolist()) == {-1, 1}
    frac = float((o.spins == 1).mean())
    assert abs(frac - 0.5) < 5 * 0.5 / math.sqrt(o.spins.size)
    for w in range(o.W):
        assert o.energies[w] == oracle.energy(8, o.spins[w])
    # the key holds the walker index: walker w is the same in any population
    o2 = oracle.OracleMuca(8, 10, 1)
    assert np.array_equal(o2.spins, o.spins[:10])
    o3 = oracle.OracleMuca(8, 10, 2)
    assert not np.array_equal(o3.spins, o2.spins)


# ---------------------------------------------------------------- thresholds
def test_thresholds_at_zero_weights():
    N = 16
    t = oracle.thresholds(N, np.zeros(N + 1))
    two32 = 1 << 32
    for k in range(N + 1):
        for d in range(5):
            kp = k + d - 2
            assert int(t[k, d]) == (two32 if 0 <= kp <= N else 0)


def test_thresholds_closed_form_values():
    N = 16
    om = np.zeros(N + 1)
    om[5] = -1.0        # moves 3->5, 4->5, 6->5, 7->5 are suppressed by e^-1
    om[9] = 25.0        # leaving bin 9 costs e^-25 < 2^-32: never accepted
    t = oracle.thresholds(N, om)
    two32 = 1 << 32
    with mpmath.workdps(50):
        want = int(mpmath.floor(mpmath.exp(-1) * two32))
    assert want == 1580030168
    assert int(t[4, 3]) == want          # k = 4 -> k' = 5
    assert int(t[3, 4]) == want          # k = 3 -> k' = 5
    assert int(t[5, 3]) == two32         # uphill in weight: always
    assert int(t[5, 2]) == two32         # Delta E = 0: always
    assert int(t[9, 1]) == 0 and int(t[9, 3]) == 0
    assert int(t[8, 3]) == two32
    # half the weight: exp(-ln 2) rounds to 1/2, floor(2^31) exactly
    om2 = np.zeros(N + 1)
    om2[7] = -math.log(2.0)
    assert int(oracle.thresholds(N, om2)[6, 3]) == 1 << 31


def test_thresholds_monotone_in_weight_drop():
    N = 16
    prev = 1 << 32
    for drop in np.linspace(0.0, 30.0, 200):
        om = np.zeros(N + 1)
        om[9] = -drop
        v = int(oracle.thresholds(N, om)[8, 3])
        assert v <= prev
        prev = v
    assert prev == 0


# ------------------------------------------------------------- weight update
def test_reweight_eq4():
    om = np.array([0.5, 1.0, -2.0, 3.0, 0.0])
    h = np.array([4, 0, 1, 10, 7], dtype=np.uint64)
    got = oracle.reweight(om, h)
    assert got[0] == 0.5 - math.log(4.0)
    assert got[1] == 1.0                  # empty bin keeps its weight
    assert got[2] == -2.0                 # ln 1 = 0
    assert got[3] == 3.0 - math.log(10.0)
    assert got[4] == 0.0 - math.log(7.0)


def test_reweight_fixed_point_at_exact_weights():
    # a histogram proportional to g e^omega is flat when omega = -ln g;
    # the update then shifts omega by one constant only.
    g = exact_dos.enumerate_dos(4)
    om = -exact_dos.ln_dos(g)
    om[~oracle.reachable_mask(16)] = 0.0
    h = np.where(oracle.reachable_mask(16), 1000, 0).astype(np.uint64)
    new = oracle.reweight(om, h)
    diff = (new - om)[oracle.reachable_mask(16)]
    assert np.max(np.abs(diff + np.log(1000.0))) < 1e-12


# ------------------------------------------------- flatness and convergence
def test_flatness():
    N = 16
    h = np.zeros(N + 1, dtype=np.uint64)
    assert oracle.flatness(h) == 0.0
    h[:] = 50
    h[1] = 0
    h[N - 1] = 0                          # forbidden bins are not counted
    assert oracle.flatness(h) == 1.0
    h[1] = 999                            # ... even when nonzero
    assert oracle.flatness(h) == 1.0
    h[4] = 20                             # sum over 15 reachable bins = 720
    assert oracle.flatness(h) == 20 / (720 / 15)


def test_chebyshev_and_kl():
    N = 16
    h = np.zeros(N + 1, dtype=np.uint64)
    h[oracle.reachable_mask(N)] = 100
    assert oracle.chebyshev(h) == 0.0
    h[6] = 250                            # m = 1650 / 15 = 110
    assert abs(oracle.chebyshev(h) - (250 / 110 - 1)) < 1e-15
    # KL of a histogram flat over w bins against Q = 1/w vanishes
    f = np.zeros(N + 1, dtype=np.uint64)
    f[2:14] = 7
    assert abs(oracle.kl_divergence(f, 12)) < 1e-15
    assert oracle.width(f) == 12
    # w is at least 10, and empty bins drop out
    f2 = np.zeros(N + 1, dtype=np.uint64)
    f2[3] = 5
    assert abs(oracle.kl_divergence(f2, 1) - math.log(10.0)) < 1e-15
    # the full range spans N + 1 bins of which N - 1 are reachable: a
    # histogram flat on the reachable bins has d_k = 0 against Q = 1/(N-1)
    full = np.zeros(N + 1, dtype=np.uint64)
    full[oracle.reachable_mask(N)] = 9
    assert oracle.width(full) == N + 1
    assert oracle.reachable_width(full) == N - 1
    assert abs(oracle.kl_divergence(full, N - 1)) < 1e-15
    # against a Q on more bins than P fills, d_k = ln(w / n) for P flat on n
    assert abs(oracle.kl_divergence(f, 24) - math.log(2.0)) < 1e-15
    assert oracle.reachable_width(f) == 12          # bins 2..13 hold no forbidden bin
    g = np.zeros(N + 1, dtype=np.uint64)
    g[[0, 2, 3]] = 4                                # range 0..3 holds forbidden bin 1
    assert oracle.width(g) == 4 and oracle.reachable_width(g) == 3



# -------------------------------------------------------------------- ln g
def test_log_dos_recovers_g_from_ideal_histogram():
    g = exact_dos.enumerate_dos(4)
    lng = exact_dos.ln_dos(g)
    h = np.array(g, dtype=np.uint64)     # the histogram at omega = 0 is g itself
    for norm in (0, 1):
        got = oracle.log_dos(h, np.zeros(17), norm)
        m = oracle.reachable_mask(16)
        assert np.max(np.abs(got[m] - lng[m])) < 1e-12
        assert np.all(np.isneginf(got[~m]))
    # weights cancel: H = g e^omega (up to rounding to integers)
    om = random_log_weights(4, 3, scale=1.0)
    h2 = np.round(np.array(g, dtype=np.float64) * np.exp(om) * 1e6).astype(np.uint64)
    got = oracle.log_dos(h2, om, 0)
    m = oracle.reachable_mask(16)
    assert np.max(np.abs(got[m] - lng[m])) < 1e-5
    assert oracle.log_dos(np.zeros(17, dtype=np.uint64), np.zeros(17), 0) is None
