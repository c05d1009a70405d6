"""The paper's iteration schedule run by the library against the oracle's
run of the same schedule: equal stop decisions, iteration counts, attempt
counts per iteration, and bit-identical weights, histograms and lattices."""
import sys

import numpy as np
import pytest

import oracle
from oracle.protocol import run_paper_schedule

pytestmark = pytest.mark.gpu

CASES = [(4, 64, 1, 400, "kl"), (6, 100, 2, 400, "kl"), (8, 64, 3, 400, "kl"), (8, 512, 4, 400, "kl"),
         (16, 128, 5, 40, "kl"), (32, 64, 6, 30, "kl"), (4, 64, 7, 400, "chebyshev"),
         (8, 512, 8, 400, "chebyshev")]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    yield


@pytest.mark.parametrize("case", CASES)
def test_schedule_matches_oracle(case):
    from paper_1707_00919_amd import Solver
    L, W, seed, cap, stop = case
    print("schedule L=%d W=%d cap=%d stop=%s" % (L, W, cap, stop), flush=True)
    sys.stdout.flush()
    g = Solver(L, W, seed)
    o = oracle.OracleMuca(L, W, seed)
    ok_g, sg = g.run_schedule(max_iterations=cap, stop=stop)
    ok_o, so = run_paper_schedule(o, max_iterations=cap, stop=stop)
    assert ok_g == ok_o
    if stop == "chebyshev":
        assert ok_g and sg[-1]["chebyshev"] < 0.05
    assert len(sg) == len(so)
    for a, b in zip(sg, so):
        assert a["therm_attempts"] == b["therm_attempts"]
        assert a["update_attempts"] == b["update_attempts"]
        assert a["width"] == b["width"] and a["covered"] == b["covered"]
        assert abs(a["kl_divergence"] - b["kl_divergence"]) <= 1e-12 * max(1.0, abs(b["kl_divergence"]))
        assert abs(a["chebyshev"] - b["chebyshev"]) <= 1e-12 * max(1.0, abs(b["chebyshev"]))
    np.testing.assert_array_equal(g.histogram(), o.hist)
    np.testing.assert_array_equal(g.log_weights().view(np.uint64), o.omega.view(np.uint64))
    np.testing.assert_array_equal(g.energies(), o.energies)
    np.testing.assert_array_equal(g.spins(), o.spins)
    assert g.last_info()["position"] == o.position
