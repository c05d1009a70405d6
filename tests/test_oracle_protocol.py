"""Pins for the oracle's run of the paper's iteration schedule (Sec. 3).

The paper prints no worked example of the schedule, so its update counts are
pinned by what they must achieve and by bookkeeping:
  * on the 4 x 4 lattice the schedule stops by its own rule (d_k < 10^-4
    after the full range is covered) and a production run at the weights it
    leaves gives ln g within 0.02 of exhaustive enumeration;
  * every attempt the schedule asks for is made: the chain position equals
    the sum of the thermalisation and update counts, and each iteration's
    histogram holds walkers * updates entries;
  * before the full range is covered the counts depend on w alone, and in
    the growth phase consecutive update counts grow by the factor 1.1.
"""
import math
import os

import numpy as np

import oracle
from oracle.protocol import run_paper_schedule


def golden_ln_g(golden_dir, L):
    with open(os.path.join(golden_dir, "ising_dos_L%d.txt" % L)) as f:
        g = [int(x) for x in f if not x.startswith("#")]
    return np.array([math.log(v) if v > 0 else -np.inf for v in g])


def test_schedule_converges_to_exact_dos(golden_dir):
    L, W = 4, 64
    o = oracle.OracleMuca(L, W, 1)
    ok, steps = run_paper_schedule(o, max_iterations=400)
    assert ok
    full = [i for i, s in enumerate(steps) if s["width"] == L * L + 1]
    assert full and steps[-1]["kl_divergence"] < 1e-4 and len(steps) - 1 >= full[0]
    assert all(s["kl_divergence"] >= 1e-4 for s in steps[full[0]:-1])
    o.production(200, 20000)
    ln_g = o.log_dos(0)
    exact = golden_ln_g(golden_dir, L)
    m = oracle.reachable_mask(L * L)
    assert np.max(np.abs(ln_g[m] - exact[m])) < 0.02


def test_chebyshev_stop_rule_converges_to_exact_dos(golden_dir):
    # App. A's alternative stop rule, d_c < 0.05 from the first full-range
    # iteration on: it ends the schedule, every earlier full-range iteration
    # had d_c >= 0.05, and the weights it leaves give ln g within 0.02
    L, W = 4, 64
    o = oracle.OracleMuca(L, W, 2)
    ok, steps = run_paper_schedule(o, max_iterations=400, stop="chebyshev")
    assert ok
    full = [i for i, s in enumerate(steps) if s["width"] == L * L + 1]
    assert full and steps[-1]["chebyshev"] < 0.05
    assert all(s["chebyshev"] >= 0.05 for s in steps[full[0]:-1])
    # d_c is the largest relative deviation from the flat mean over the
    # reachable bins of the last histogram
    h = o.hist.astype(float)
    m = oracle.reachable_mask(L * L)
    mean = h[m].sum() / m.sum()
    assert abs(np.max(np.abs(h[m] / mean - 1.0)) - steps[-1]["chebyshev"]) < 1e-12
    o.production(200, 20000)
    exact = golden_ln_g(golden_dir, L)
    assert np.max(np.abs(o.log_dos(0)[m] - exact[m])) < 0.02


def test_schedule_bookkeeping():
    L, W = 6, 40
    o = oracle.OracleMuca(L, W, 3)
    pos = 0
    ok, steps = run_paper_schedule(o, max_iterations=30)
    for s in steps:
        pos += s["therm_attempts"] + s["update_attempts"]
        assert s["therm_attempts"] == 30 * s["width"]
        assert s["width"] >= 10
    assert o.position == pos
    assert int(o.hist.sum()) == W * steps[-1]["update_attempts"]


def test_schedule_counts_follow_w_then_grow():
    L, W = 6, 64
    o = oracle.OracleMuca(L, W, 5)
    ok, steps = run_paper_schedule(o, max_iterations=60)
    first_full = next(i for i, s in enumerate(steps) if s["width"] == L * L + 1)
    by_w = {}
    for s in steps[:first_full + 1]:
        by_w.setdefault(s["width"], set()).add(s["update_attempts"])
    assert all(len(v) == 1 for v in by_w.values())
    grow = [s["update_attempts"] for s in steps[first_full:]]
    for a, b in zip(grow, grow[1:]):
        # b - 1 = floor(1.1 x), a - 1 = floor(x): |b - 1 - 1.1 (a - 1)| < 1.1
        assert abs((b - 1) - 1.1 * (a - 1)) < 1.1 + 1e-9
