"""Seeded synthetic inputs shared by the tests, the oracle and the benchmark.

This module holds workload shapes and seeded random inputs only -- none of
the method's arithmetic.  The multicanonical chain draws its own random
numbers (Philox4x32-10, keyed by seed and walker), so an input here is just
(L, walkers, seed) plus, where a test needs a nonzero weight table, a seeded
log-weight array omega[k], k = 0..L*L.

The paper's workload is the 2D Ising model itself (Sec. 3): no dataset is
involved.  The named workloads below are the sizes the paper works at
(L = 16, 32, 64 with O(10^4) walkers, Sec. 3.1) plus the small case an
exhaustive enumeration can check.
"""
import numpy as np

# Named workloads.  iter_sweeps: recorded sweeps per weight iteration;
# iterations: fixed count (None = until flatness >= min_flat);
# prod_sweeps: recorded sweeps of the final production run, preceded by
# prod_therm_sweeps unrecorded sweeps at the final weights (the walkers start
# the production in equilibrium with the previous weights only);
# therm_sweeps: unrecorded sweeps before each weight iteration.
WORKLOADS = {
    "ising_L4_W64": dict(L=4, walkers=64, iter_sweeps=2000, iterations=8, min_flat=None,
                         prod_sweeps=20000, prod_therm_sweeps=0, therm_sweeps=0),
    "ising_L32_W16384": dict(L=32, walkers=16384, iter_sweeps=200, iterations=None,
                             min_flat=0.5, prod_sweeps=10000, prod_therm_sweeps=10000,
                             therm_sweeps=0),
    "ising_L64_W65536": dict(L=64, walkers=65536, iter_sweeps=500, iterations=None,
                             min_flat=0.5, prod_sweeps=10000, prod_therm_sweeps=10000,
                             therm_sweeps=0),
    "ising_L128_W16384": dict(L=128, walkers=16384, iter_sweeps=500, iterations=None,
                              min_flat=0.5, prod_sweeps=10000, prod_therm_sweeps=10000,
                              therm_sweeps=0),
}


def random_log_weights(L, seed, scale=2.0):
    """Independent uniform log weights in [-scale, scale] for every bin."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=L * L + 1).astype(np.float64)


def smooth_log_weights(L, seed, depth=None):
    """A smooth, bowl-shaped random log-weight profile of the kind a weight
    iteration produces: low in the middle of the energy range, high at the
    edges (depth ~ N ln 2 by default), plus a seeded low-frequency wiggle."""
    N = L * L
    rng = np.random.default_rng(seed)
    if depth is None:
        depth = 0.6 * N
    u = np.linspace(-1.0, 1.0, N + 1)
    bowl = depth * (u * u - 1.0)
    wiggle = np.zeros(N + 1)
    for m in range(1, 5):
        wiggle += rng.normal(0.0, 1.0) * np.sin(np.pi * m * (u + 1.0) / 2.0)
    return (bowl + wiggle).astype(np.float64)


def parity_cases():
    """(L, walkers, seed) triples for GPU-vs-oracle parity: several tiles,
    ragged walker counts, and every lattice-shape class (L mod 4, L mod 32)."""
    return [
        (4, 64, 1), (4, 1, 7), (6, 65, 2), (8, 63, 3), (10, 100, 4), (12, 130, 5),
        (16, 64, 6), (16, 257, 7), (24, 96, 8), (30, 70, 9), (32, 128, 10), (32, 4097, 11),
        (34, 66, 12), (48, 80, 13), (64, 64, 14), (128, 65, 15),
    ]


# The batched workload: 48 independent instances of uneven size.  L is drawn
# uniformly from BATCH_LS, then the walker counts log-uniformly on
# [256, 8192] (rounded, no alignment), both from default_rng(0); instance i
# has seed i + 1.  Every instance runs weight iterations of 200 sweeps until
# its flatness reaches 0.5 (or the iteration cap), then a 2000-sweep
# production run preceded by 2000 unrecorded sweeps.
BATCH_LS = (8, 12, 16, 24, 32, 48, 64)
BATCH_WORKLOAD = dict(instances=48, iter_sweeps=200, min_flat=0.5, max_iterations=400,
                      prod_sweeps=2000, prod_therm_sweeps=2000)


def batch_instances(count=48, rng_seed=0):
    """[(L, walkers, seed)] of the batched workload."""
    rng = np.random.default_rng(rng_seed)
    Ls = rng.choice(np.array(BATCH_LS), size=count)
    walkers = np.rint(np.exp(rng.uniform(np.log(256.0), np.log(8192.0), size=count))).astype(int)
    return [(int(L), int(W), i + 1) for i, (L, W) in enumerate(zip(Ls, walkers))]


# The serving workload: Poisson arrivals at SERVE_RATE requests/s for
# SERVE_DURATION s from default_rng(1) (exponential gaps, then per request L
# uniform from SERVE_LS and walkers log-uniform on [1024, 16384]); request i
# has seed 1000 + i.  Each request iterates with 200-sweep iterations to
# flatness 0.5, then runs 2000 unrecorded and 2000 recorded production sweeps.
SERVE_LS = (16, 24, 32, 48, 64)
SERVE_RATE = 20.0
SERVE_DURATION = 60.0
SERVE_REQUEST = dict(iter_sweeps=200, min_flatness=0.5, max_iterations=2000, prod_therm=2000,
                     prod_sweeps=2000)


def serving_requests(rate=SERVE_RATE, duration=SERVE_DURATION, rng_seed=1):
    """[(arrival_s, L, walkers, seed)] of the serving workload."""
    rng = np.random.default_rng(rng_seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        L = int(rng.choice(np.array(SERVE_LS)))
        W = int(np.rint(np.exp(rng.uniform(np.log(1024.0), np.log(16384.0)))))
        out.append((t, L, W, 1000 + len(out)))
    return out
