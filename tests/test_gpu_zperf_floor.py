"""A floor on the sweep rate, kept in a file that runs after the correctness
tests (a slow device must not hide them).

The sweep rate at L = 32 with 16384 walkers at the exact weights (the paper's
hardware measurement, Sec. 3.1) stays above 3.0e11 attempts/s, about three
quarters of what the kernel reaches on an MI355X (4.1e11): a guard against a
performance regression, not a measurement (bench.py measures).
"""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    yield


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def exact_ln_g(L):
    with open(os.path.join(GOLDEN, "ising_dos_L%d.txt" % L)) as f:
        g = [int(x) for x in f if not x.startswith("#")]
    return np.array([math.log(v) if v > 0 else -np.inf for v in g])


def test_sweep_rate_floor_at_the_papers_scale():
    from paper_1707_00919_amd import Solver
    note("sweep rate floor L=32 W=16384")
    L, W = 32, 16384
    lng = exact_ln_g(L)
    s = Solver(L, W, 12345)
    s.set_log_weights(np.where(np.isfinite(lng), -lng, 0.0))
    s.production(0, 20)
    info = s.production(0, 200)
    rate = info["attempts"] / (info["kernel_ms"] * 1e-3)
    note("  %.3e attempts/s (kernel variant %d)" % (rate, info["kernel_variant"]))
    assert rate > 3.0e11
    s.close()
