"""Production analysis on GPU data: a production run in 100 blocks at the
exact weights, jackknife error bars on ln g, canonical averages.

  * the block histograms sum, bit for bit, to the histogram of one
    production call of the same length on a twin instance;
  * ln g agrees with the exact result within the stated 0.02, and the
    deviations are consistent with the jackknife errors;
  * the reweighted <E>/N and C/N agree with their exact values within a few
    jackknife errors.
"""
import math
import os
import sys

import numpy as np
import pytest

from oracle import analysis as A

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    yield


def exact_ln_g(L):
    path = os.path.join(os.path.dirname(__file__), "golden", "ising_dos_L%d.txt" % L)
    with open(path) as f:
        g = [int(x) for x in f if not x.startswith("#")]
    return np.array([math.log(v) if v > 0 else -np.inf for v in g])


def test_blocks_jackknife_and_canonical():
    from paper_1707_00919_amd import Solver, analysis
    L, W, seed = 16, 4096, 3
    print("analysis L=%d W=%d" % (L, W), flush=True)
    sys.stdout.flush()
    lng = exact_ln_g(L)
    omega = np.where(np.isfinite(lng), -lng, 0.0)
    a = Solver(L, W, seed)
    b = Solver(L, W, seed)
    for s in (a, b):
        s.set_log_weights(omega)
    blocks = analysis.production_blocks(a, 200, 20, 100)
    b.production(200, 2000)
    np.testing.assert_array_equal(blocks.sum(axis=0, dtype=np.uint64), b.histogram())

    est, err = analysis.jackknife_log_dos(L, blocks, omega, 1)
    m = np.isfinite(lng)
    dev = np.abs(est[m] - lng[m])
    assert dev.max() < 0.02
    assert np.all(np.isfinite(err[m]))
    assert np.mean(dev < 3 * err[m]) > 0.9

    betas = [0.3, 0.4406867935, 0.6]
    e, ee, c, ce = analysis.canonical(L, blocks, omega, betas)
    ex, cx = A.canonical(lng, betas)
    assert np.all(np.abs(e - ex) < 5 * ee + 1e-12)
    assert np.all(np.abs(c - cx) < 5 * ce + 1e-12)
