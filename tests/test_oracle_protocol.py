"""Pins for the oracle's run of the paper's iteration schedule (Sec. 3).

The paper prints no worked example of the schedule.  Its update counts are
pinned by Eq. 7 worked by hand (the literal counts at the end of this file,
for two walker counts, before and after the full range is reached), by what
they must achieve and by bookkeeping:
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


# Eq. 7 worked by hand for the 6 x 6 lattice (N + 1 = 37 bins, so the full
# range is w = 37).  x = 6 w^2.25 / W, N_updates = floor(x) + 1:
#   W = 64: w = 10: 10^2.25 = 177.8279..., x = 6 * 177.8279 / 64 = 16.671 -> 17
#           w = 16: 16^2.25 = 2^9 = 512, x = 3072 / 64 = 48 exactly   -> 49
#           w = 37: 37^2.25 = 3376.40..., x = 316.537                 -> 317
#   W = 40: w = 10: x = 26.674 -> 27; w = 16: x = 76.8 -> 77; w = 37: x = 506.460 -> 507
# (w^2.25 = exp(2.25 ln w); the values for the other w were worked the same way,
# to 50 digits, and are listed below).  After the first full-range iteration x
# grows by 1.1 per iteration:
#   W = 64: 316.537 * 1.1 = 348.191 -> 349, 383.010 -> 384, 421.311 -> 422, 463.443 -> 464
#   W = 40: 506.460 * 1.1 = 557.106 -> 558, 612.817 -> 613, 674.098 -> 675, 741.508 -> 742
# N_therm = f_therm * w = 30 w attempts per walker.
EQ7_COUNTS = {
    64: dict(zip(range(10, 38), [17, 21, 26, 31, 36, 42, 49, 56, 63, 71, 80, 89, 99, 109, 120, 132,
                                 144, 156, 170, 183, 198, 213, 229, 245, 262, 280, 298, 317])),
    40: dict(zip(range(10, 38), [27, 34, 41, 49, 57, 67, 77, 89, 101, 114, 127, 142, 158, 174, 192, 210,
                                 229, 250, 271, 293, 316, 341, 366, 392, 419, 447, 477, 507])),
}
EQ7_GROWTH = {64: [349, 384, 422, 464], 40: [558, 613, 675, 742]}


def test_schedule_counts_equal_eq7_worked_by_hand():
    L = 6
    for W, seed in ((64, 5), (40, 3)):
        o = oracle.OracleMuca(L, W, seed)
        ok, steps = run_paper_schedule(o, max_iterations=60)
        assert steps[0]["width"] == 10 and steps[0]["update_attempts"] == EQ7_COUNTS[W][10]
        assert steps[0]["therm_attempts"] == 300
        first_full = next(i for i, s in enumerate(steps) if s["width"] == L * L + 1)
        for s in steps[:first_full + 1]:
            assert s["update_attempts"] == EQ7_COUNTS[W][s["width"]], (W, s)
            assert s["therm_attempts"] == 30 * s["width"]
        assert steps[first_full]["update_attempts"] == EQ7_COUNTS[W][37]
        grown = [s["update_attempts"] for s in steps[first_full + 1:first_full + 5]]
        assert len(grown) == 4, "the schedule stopped before four growth iterations"
        assert grown == EQ7_GROWTH[W]
