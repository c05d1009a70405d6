"""Pins for the exact density of states (the paper's ground truth, Sec. 3).

The Kaufman closed form is checked against two independent counts
(brute-force enumeration at L = 4, the transfer matrix at L = 4, 6) and
against closed-form counts of the lowest excitations that follow from
drawing the flipped clusters by hand:

  g(E_min)      = 2                  two ground states (Sec. 3.3)
  g(E_min + 4)  = 0                  forbidden (Sec. 3)
  g(E_min + 8)  = 2N                 one flipped spin
  g(E_min + 12) = 4N                 a flipped domino (two orientations)
  g(E_min + 16) = N(N-1) + 10N       two separated single flips, straight and
                                     bent trimers, 2x2 squares (L >= 6)
"""
import math
import os

import numpy as np

import pytest

from oracle import exact_dos

SIZES = [4, 6, 8, 12, 16, 24, 32]


def load(golden_dir, L):
    path = os.path.join(golden_dir, "ising_dos_L%d.txt" % L)
    if not os.path.exists(path):
        pytest.skip("golden table for L=%d not generated" % L)
    with open(path) as f:
        return [int(line) for line in f if not line.startswith("#")]


def test_enumeration_matches_kaufman_L4(golden_dir):
    g = exact_dos.enumerate_dos(4)
    assert g == exact_dos.kaufman_dos(4)
    assert g == load(golden_dir, 4)
    # the L = 4 table, energies -32..32 in steps of 4
    assert g == [2, 0, 32, 64, 424, 1728, 6688, 13568, 20524, 13568, 6688, 1728, 424, 64,
                 32, 0, 2]


@pytest.mark.parametrize("L", [4, 6])
def test_transfer_matrix_matches_kaufman(L, golden_dir):
    assert exact_dos.transfer_matrix_dos(L) == exact_dos.kaufman_dos(L) == load(golden_dir, L)


def test_kaufman_live_matches_golden_L8(golden_dir):
    assert exact_dos.kaufman_dos(8) == load(golden_dir, 8)


@pytest.mark.parametrize("L", SIZES)
def test_golden_invariants(L, golden_dir):
    g = load(golden_dir, L)
    N = L * L
    assert len(g) == N + 1
    assert sum(g) == 2 ** N
    assert g == g[::-1]                      # E -> -E on a bipartite torus
    assert g[0] == 2 and g[1] == 0 and g[N - 1] == 0
    assert g[2] == 2 * N
    assert g[3] == 4 * N
    if L >= 6:
        assert g[4] == N * (N - 1) + 10 * N
    assert all(v > 0 for k, v in enumerate(g) if k not in (1, N - 1))


def test_ln_dos_helper():
    g = exact_dos.enumerate_dos(4)
    ln = exact_dos.ln_dos(g)
    assert ln[1] == float("-inf")
    assert abs(ln[8] - 9.9293502) < 1e-6    # ln 20524


def test_golden_log_table_L64(golden_dir):
    # the L = 64 table holds ln g (the integers run to 1233 digits): the same
    # hand-counted low-energy values, the E <-> -E symmetry and the total 2^N
    path = os.path.join(golden_dir, "ising_lndos_L64.txt")
    with open(path) as f:
        lng = np.array([float(x) for x in f if not x.startswith("#")])
    L, N = 64, 64 * 64
    assert lng.size == N + 1
    assert np.array_equal(lng, lng[::-1])
    assert lng[0] == math.log(2) and lng[1] == -np.inf and lng[N - 1] == -np.inf
    assert abs(lng[2] - math.log(2 * N)) < 1e-15 * math.log(2 * N)
    assert abs(lng[3] - math.log(4 * N)) < 1e-15 * math.log(4 * N)
    assert abs(lng[4] - math.log(N * (N - 1) + 10 * N)) < 1e-14
    fin = np.isfinite(lng)
    assert fin.sum() == N - 1
    mx = lng[fin].max()
    total = mx + math.log(np.exp(lng[fin] - mx).sum())
    assert abs(total - N * math.log(2)) < 1e-9 * N
