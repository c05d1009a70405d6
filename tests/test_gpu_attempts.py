"""Calls counted in attempts (they start and stop inside sweeps) against the
oracle, bit for bit: every histogram, then spins, energies and weights.

The call sequences cross sweep boundaries, start recording inside a sweep,
run fewer attempts than one row, whole sweeps from an unaligned position,
and zero attempts; each shape runs with the fast-layout and the generic
threshold tables.
"""
import sys

import numpy as np
import pytest

import oracle
from muca_inputs import random_log_weights

pytestmark = pytest.mark.gpu

SHAPES = [(4, 64, 21), (6, 70, 22), (8, 100, 23), (16, 65, 24), (34, 64, 25), (64, 64, 26),
          (80, 64, 27), (128, 64, 28)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    yield


def calls(N, rng):
    """(kind, therm, count): kind 'a' = attempts, 's' = sweeps."""
    seq = [("a", 0, 1), ("a", 3, N - 5), ("a", N + 2, 2 * N + 7), ("a", 0, 0), ("s", 1, 2),
           ("a", 5, 0), ("a", 0, N), ("a", int(rng.integers(0, 3 * N)), int(rng.integers(1, 3 * N))),
           ("a", (N - 3 - 5 - 2 * N - 7 - 5) % N, 2 * N), ("s", 0, 1)]
    return seq


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("shape", SHAPES)
def test_attempt_calls_match_oracle(shape, generic):
    from paper_1707_00919_amd import Solver, _abi
    L, W, seed = shape
    N = L * L
    print("attempt calls L=%d W=%d generic=%d" % (L, W, generic), flush=True)
    sys.stdout.flush()
    flags = _abi.MUCA_FLAG_GENERIC_KERNEL if generic else 0
    g = Solver(L, W, seed, flags=flags)
    o = oracle.OracleMuca(L, W, seed)
    om = random_log_weights(L, seed, scale=1.5)
    g.set_log_weights(om)
    o.set_log_weights(om)
    rng = np.random.default_rng(seed)
    for i, (kind, th, n) in enumerate(calls(N, rng)):
        update = i % 2 == 0
        if kind == "a":
            gi = (g.iterate_attempts if update else g.production_attempts)(th, n)
            oi = (o.iterate_attempts if update else o.production_attempts)(th, n)
        else:
            gi = (g.iterate if update else g.production)(th, n)
            oi = (o.iterate if update else o.production)(th, n)
        np.testing.assert_array_equal(g.histogram(), o.hist, err_msg="call %d" % i)
        assert gi["position"] == oi["position"] == o.position
        assert gi["sweep_counter"] == oi["sweep_counter"]
        assert gi["hist_sum"] == oi["hist_sum"]
    np.testing.assert_array_equal(g.energies(), o.energies)
    np.testing.assert_array_equal(g.spins(), o.spins)
    np.testing.assert_array_equal(g.log_weights().view(np.uint64), o.omega.view(np.uint64))


def test_batch_refuses_unaligned_member():
    from paper_1707_00919_amd import Batch, MucaError, Solver, _abi
    a, b = Solver(8, 64, 1), Solver(8, 64, 2)
    a.iterate_attempts(0, 10)
    batch = Batch([a, b])
    with pytest.raises(MucaError) as e:
        batch.run([1, 1], [0, 0], [1, 1])
    assert e.value.code == _abi.MUCA_ERR_INVALID_ARG
    a.iterate_attempts(0, 64 - 10)      # back on a sweep boundary
    batch.run([1, 1], [0, 0], [1, 1])
