"""GPU parity: libmuca (HIP kernels for gfx950, called through the C ABI)
against the CPU oracle, element by element and bit-exactly.

Compared after every call: the spins and energy of every walker, the merged
histogram, the threshold table, the log weights (bit patterns), the sweep
counter and the histogram statistics.  Cases cover several waves and ragged
walker counts, every lattice-shape class (L mod 4, one to four 32-bit words
per row, thresholds in LDS or in L2), the small workload end to end, and the
full-size shapes of the benchmark (L = 32 with 16384 walkers, L = 64 with
65536, L = 128 with 16384) over a few sweeps, in the launch configuration the
benchmark times.
"""
import sys

import numpy as np
import pytest

import oracle
from muca_inputs import parity_cases, random_log_weights, smooth_log_weights
from oracle import exact_dos

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_1707_00919_amd
    paper_1707_00919_amd.lib()
    yield


def Solver(*a, **kw):
    from paper_1707_00919_amd import Solver as S
    return S(*a, **kw)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def assert_state(s, o):
    np.testing.assert_array_equal(s.energies(), o.energies)
    np.testing.assert_array_equal(s.spins(), o.spins)


def assert_call(si, oi, s, o):
    np.testing.assert_array_equal(s.histogram(), o.hist)
    np.testing.assert_array_equal(s.thresholds(), o.table)
    np.testing.assert_array_equal(bits(s.log_weights()), bits(o.omega))
    assert si["sweep_counter"] == o.sweep_counter
    assert si["hist_sum"] == oi["hist_sum"]
    assert si["attempts"] == oi["attempts"]
    assert si["visited_bins"] == oi["visited_bins"]
    assert si["flatness"] == oi["flatness"]
    assert abs(si["kl_divergence"] - oi["kl_divergence"]) <= 1e-12 * max(1.0, abs(oi["kl_divergence"]))
    assert abs(si["chebyshev"] - oi["chebyshev"]) <= 1e-12 * max(1.0, abs(oi["chebyshev"]))


@pytest.mark.parametrize("L,W,seed", parity_cases())
def test_init_matches_oracle(L, W, seed):
    note("init L=%d W=%d seed=%d" % (L, W, seed))
    s = Solver(L, W, seed)
    o = oracle.OracleMuca(L, W, seed)
    assert_state(s, o)
    np.testing.assert_array_equal(s.thresholds(), o.table)


@pytest.mark.parametrize("L,W,seed", parity_cases())
def test_sweeps_match_oracle(L, W, seed):
    note("sweeps L=%d W=%d seed=%d" % (L, W, seed))
    s = Solver(L, W, seed)
    o = oracle.OracleMuca(L, W, seed)
    om = random_log_weights(L, seed, scale=2.0)
    s.set_log_weights(om)
    o.set_log_weights(om)
    assert_call(s.production(2, 3), o.production(2, 3), s, o)
    assert_state(s, o)
    om2 = smooth_log_weights(L, seed)
    s.set_log_weights(om2)
    o.set_log_weights(om2)
    for _ in range(2):
        assert_call(s.iterate(1, 2), o.iterate(1, 2), s, o)
        assert_state(s, o)


def test_small_workload_end_to_end():
    # L = 4, 64 walkers: 8 weight iterations x 2000 sweeps, then 20000
    # production sweeps, bit-exact at every step; ln g within 0.02 of the
    # exhaustive enumeration.
    note("small workload L=4 W=64 seed=1")
    s = Solver(4, 64, 1)
    o = oracle.OracleMuca(4, 64, 1)
    for _ in range(8):
        assert_call(s.iterate(0, 2000), o.iterate(0, 2000), s, o)
    assert_call(s.production(0, 20000), o.production(0, 20000), s, o)
    assert_state(s, o)
    for norm in (0, 1):
        np.testing.assert_array_equal(bits(s.log_dos(norm)), bits(o.log_dos(norm)))
    exact = exact_dos.ln_dos(exact_dos.enumerate_dos(4))
    m = oracle.reachable_mask(16)
    assert np.max(np.abs(s.log_dos(0)[m] - exact[m])) < 0.02


@pytest.mark.parametrize("L,W,seed", [(4, 64, 1), (6, 65, 2), (16, 257, 7), (30, 70, 9),
                                      (32, 4097, 11), (34, 66, 12), (48, 80, 13), (62, 65, 3),
                                      (64, 64, 14), (40, 200, 15), (44, 65, 16), (56, 130, 17),
                                      (64, 320, 18), (48, 192, 19),
                                      # two-wave loop steps of four rows (L = 8 ... 28) and
                                      # of two rows (L = 36, 52, 60)
                                      (8, 65, 20), (12, 64, 21), (20, 66, 22), (24, 70, 23),
                                      (28, 130, 24), (36, 65, 25), (52, 64, 26), (60, 65, 27)])
def test_kernel_variants_agree(L, W, seed):
    # split (two waves, thresholds fetched ahead), fast (one wave) and generic
    # (64-bit thresholds) sweep kernels: the same bits, and the oracle's
    from paper_1707_00919_amd import _abi
    note("kernel variants L=%d W=%d seed=%d" % (L, W, seed))
    o = oracle.OracleMuca(L, W, seed)
    runs = [(Solver(L, W, seed), 2 if L != 62 else 1),
            (Solver(L, W, seed, flags=_abi.MUCA_FLAG_FAST_KERNEL), 1),
            (Solver(L, W, seed, flags=_abi.MUCA_FLAG_GENERIC_KERNEL), 0)]
    om = smooth_log_weights(L, seed + 100)
    o.set_log_weights(om)
    oi = o.iterate(2, 3)
    for s, variant in runs:
        s.set_log_weights(om)
        si = s.iterate(2, 3)
        assert si["kernel_variant"] == variant
        assert_call(si, oi, s, o)
        assert_state(s, o)


@pytest.mark.parametrize("L,extra,trim,seed", [(48, 1, 0, 61), (52, 2, 5, 62), (56, 1, 63, 63), (64, 1, 0, 64),
                                             (64, 2, 1, 65)])
def test_pair_form_matches_oracle(L, extra, trim, seed):
    # more 64-walker blocks than CUs where one two-wave workgroup fills a CU:
    # the pair form (two chains sharing one table, whole-row steps at L = 48,
    # 52, 56 and half-row steps at L = 64); an odd block count leaves the last
    # pair's second chain idle; against the oracle and the one-wave form
    import torch
    from paper_1707_00919_amd import _abi
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    W = 64 * (cus + extra) - trim
    note("pair form L=%d W=%d seed=%d" % (L, W, seed))
    o = oracle.OracleMuca(L, W, seed)
    om = smooth_log_weights(L, seed + 100)
    o.set_log_weights(om)
    oi = o.iterate(2, 3)
    for flags, variant in [(0, 5), (_abi.MUCA_FLAG_FAST_KERNEL, 1)]:
        s = Solver(L, W, seed, flags=flags)
        s.set_log_weights(om)
        si = s.iterate(2, 3)
        assert si["kernel_variant"] == variant
        assert_call(si, oi, s, o)
        assert_state(s, o)


@pytest.mark.parametrize("L,W,seed,default", [(80, 65, 31, 4), (96, 130, 32, 4), (112, 64, 33, 4),
                                              (128, 200, 34, 4), (96, 16448, 36, 3)])
def test_wide_kernel_agrees(L, W, seed, default):
    # L > 64: the wide kernels (thresholds from global memory, counters in
    # LDS) in their two-wave form (chosen while every workgroup is resident at
    # once) and one-wave form, and the generic kernel, against the oracle
    from paper_1707_00919_amd import _abi
    note("wide kernel L=%d W=%d seed=%d" % (L, W, seed))
    o = oracle.OracleMuca(L, W, seed)
    om = smooth_log_weights(L, seed + 100)
    o.set_log_weights(om)
    oi = o.iterate(1, 2)
    for flags, variant in [(0, default), (_abi.MUCA_FLAG_FAST_KERNEL, 3), (_abi.MUCA_FLAG_GENERIC_KERNEL, 0)]:
        s = Solver(L, W, seed, flags=flags)
        s.set_log_weights(om)
        si = s.iterate(1, 2)
        assert si["kernel_variant"] == variant
        assert_call(si, oi, s, o)
        assert_state(s, o)


def test_many_walkers_at_large_L_use_wave_groups():
    # more two-wave chains than fit on the device at once, even two per CU:
    # the one-wave form runs, with four waves sharing one record table at
    # L = 64
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    L, W, seed = 64, 64 * (2 * cus + 1), 20
    note("wave groups L=%d W=%d" % (L, W))
    s = Solver(L, W, seed)
    o = oracle.OracleMuca(L, W, seed)
    om = smooth_log_weights(L, seed)
    s.set_log_weights(om)
    o.set_log_weights(om)
    si = s.iterate(1, 1)
    oi = o.iterate(1, 1)
    assert si["kernel_variant"] == 1
    assert_call(si, oi, s, o)
    assert_state(s, o)


def test_zero_threshold_falls_back_to_generic_kernel():
    # a weight drop of 30 between neighbouring bins makes a reachable
    # threshold 0, which the 32-bit form cannot hold: the call must run the
    # generic kernel and still match the oracle
    note("zero-threshold fallback")
    L, W, seed = 8, 64, 4
    om = random_log_weights(L, 4, scale=1.0)
    om[30:] -= 30.0
    s = Solver(L, W, seed)
    o = oracle.OracleMuca(L, W, seed)
    s.set_log_weights(om)
    o.set_log_weights(om)
    assert oracle.thresholds(L * L, om)[29, 3] == 0
    si = s.production(1, 3)
    assert si["kernel_variant"] == 0
    assert_call(si, o.production(1, 3), s, o)
    assert_state(s, o)


def test_forbidden_bins_do_not_disable_the_fast_kernels():
    # the forbidden bins keep omega = 0 while their neighbours sink far below:
    # their thresholds are 0, but no configuration ever has those energies
    note("forbidden-bin thresholds")
    L, W, seed = 16, 130, 6
    N = L * L
    om = smooth_log_weights(L, 5) - 400.0
    om[1] = 0.0
    om[N - 1] = 0.0
    assert oracle.thresholds(N, om)[1, 4] == 0
    s = Solver(L, W, seed)
    o = oracle.OracleMuca(L, W, seed)
    s.set_log_weights(om)
    o.set_log_weights(om)
    si = s.iterate(1, 3)
    assert si["kernel_variant"] == 2
    assert_call(si, o.iterate(1, 3), s, o)
    assert_state(s, o)


@pytest.mark.parametrize("cap", [1, 3])
def test_launch_split_does_not_change_results(cap):
    note("launch split cap=%d" % cap)
    L, W, seed = 16, 130, 3
    om = smooth_log_weights(L, 9)
    a = Solver(L, W, seed)
    b = Solver(L, W, seed, flags=cap)
    for x in (a, b):
        x.set_log_weights(om)
    ia = a.iterate(2, 5)
    ib = b.iterate(2, 5)
    assert ib["kernel_launches"] == -(-7 // cap) and ia["kernel_launches"] == 1
    np.testing.assert_array_equal(a.histogram(), b.histogram())
    np.testing.assert_array_equal(a.spins(), b.spins())
    np.testing.assert_array_equal(a.energies(), b.energies())


def test_library_stream_and_memory_match_torch_ones():
    note("own stream/workspace vs torch")
    om = random_log_weights(12, 4)
    a = Solver(12, 200, 8, use_torch=True)
    b = Solver(12, 200, 8, use_torch=False)
    for x in (a, b):
        x.set_log_weights(om)
        x.iterate(1, 4)
    np.testing.assert_array_equal(a.histogram(), b.histogram())
    np.testing.assert_array_equal(a.spins(), b.spins())


def test_zero_sweeps_and_therm_only():
    note("zero sweeps")
    s = Solver(8, 64, 2)
    o = oracle.OracleMuca(8, 64, 2)
    om = random_log_weights(8, 2)
    s.set_log_weights(om)
    o.set_log_weights(om)
    assert_call(s.iterate(0, 0), o.iterate(0, 0), s, o)
    assert_call(s.iterate(3, 0), o.iterate(3, 0), s, o)
    assert not s.histogram().any()
    assert_state(s, o)


def _energy_from_spins(spins, L):
    sp = spins.reshape(-1, L, L).astype(np.int32)
    return -(sp * (np.roll(sp, -1, axis=2) + np.roll(sp, -1, axis=1))).sum(axis=(1, 2))


@pytest.mark.parametrize("L,W,sweeps", [(32, 16384, 2), (64, 65536, 1), (128, 16384, 1)])
def test_full_size_shapes_bit_exact(L, W, sweeps):
    # the benchmark's shapes, every walker, a few sweeps at bowl-shaped weights
    note("full size L=%d W=%d sweeps=%d" % (L, W, sweeps))
    seed = 1
    s = Solver(L, W, seed)
    o = oracle.OracleMuca(L, W, seed)
    om = smooth_log_weights(L, 21)
    s.set_log_weights(om)
    o.set_log_weights(om)
    assert_call(s.production(1, sweeps), o.production(1, sweeps), s, o)
    assert_state(s, o)
    np.testing.assert_array_equal(_energy_from_spins(s.spins(), L), s.energies())


def test_full_size_L32_two_weight_iterations():
    note("full size L=32 W=16384 two iterations")
    s = Solver(32, 16384, 7)
    o = oracle.OracleMuca(32, 16384, 7)
    for _ in range(2):
        assert_call(s.iterate(0, 3), o.iterate(0, 3), s, o)
    assert_state(s, o)


def test_headline_seed1_first_three_weight_iterations():
    # the paper-scale workload exactly as the benchmark runs it: L = 32, 16384
    # walkers, seed 1, omega = 0 at the start, 200-sweep weight iterations
    # (Sec. 3.1 scale; Eq. 4 after each); histogram, threshold table, omega
    # bits, spins and energies of every walker equal the oracle's after each
    # of the first three iterations
    from muca_inputs import WORKLOADS
    wl = WORKLOADS["ising_L32_W16384"]
    L, W = wl["L"], wl["walkers"]
    s = Solver(L, W, 1)
    o = oracle.OracleMuca(L, W, 1)
    for it in range(3):
        note("headline L=32 W=16384 seed 1, iteration %d of 200 sweeps" % (it + 1))
        assert_call(s.iterate(wl["therm_sweeps"], wl["iter_sweeps"]),
                    o.iterate(wl["therm_sweeps"], wl["iter_sweeps"]), s, o)
        assert_state(s, o)


def test_invalid_arguments_are_reported():
    from paper_1707_00919_amd import MucaError, _abi
    note("error paths")
    s = Solver(8, 64, 1)
    bad = np.zeros(65)
    bad[3] = np.nan
    with pytest.raises(MucaError) as e:
        s.set_log_weights(bad)
    assert e.value.code == _abi.MUCA_ERR_INVALID_ARG
    with pytest.raises(MucaError) as e:
        s.set_log_weights(np.zeros(64))
    assert e.value.code == _abi.MUCA_ERR_INVALID_ARG
    # the instance is still usable after argument errors
    s.iterate(0, 1)
    with pytest.raises(MucaError) as e:
        Solver(128, 1 << 30, 1, use_torch=False)   # 2 TiB of lattices
    assert e.value.code == _abi.MUCA_ERR_OUT_OF_MEMORY
    with pytest.raises(MucaError) as e:
        s.log_dos(0)   # histogram of one sweep from omega = 0 misses the ground state
    assert e.value.code == _abi.MUCA_ERR_NOT_CONVERGED


@pytest.mark.parametrize("L,W,seed", [(8, 100, 41), (32, 130, 42), (128, 64, 43)])
def test_checkpoint_resume_continues_bit_exactly(L, W, seed):
    # S1 + S2 attempts with a checkpoint/restore into a fresh instance between
    # them equal the same run without one, and the oracle's run of S1 + S2
    # (calls cut inside a sweep too)
    note("checkpoint L=%d W=%d" % (L, W))
    from paper_1707_00919_amd import MucaError, _abi
    N = L * L
    om = smooth_log_weights(L, seed)
    a, c = Solver(L, W, seed), Solver(L, W, seed)
    o = oracle.OracleMuca(L, W, seed)
    for x in (a, c, o):
        x.set_log_weights(om)
    a.iterate(1, 2)
    a.production_attempts(3, N + 7)
    state = a.checkpoint()
    b = Solver(L, W, seed)
    b.restore(state)
    a.iterate_attempts(0, 2 * N - 3)
    b.iterate_attempts(0, 2 * N - 3)
    c.iterate(1, 2)
    c.production_attempts(3, N + 7)
    c.iterate_attempts(0, 2 * N - 3)
    o.iterate(1, 2)
    o.production_attempts(3, N + 7)
    o.iterate_attempts(0, 2 * N - 3)
    for s in (a, b, c):
        np.testing.assert_array_equal(s.histogram(), o.hist)
        np.testing.assert_array_equal(bits(s.log_weights()), bits(o.omega))
        np.testing.assert_array_equal(s.energies(), o.energies)
        np.testing.assert_array_equal(s.spins(), o.spins)
        assert s.last_info()["position"] == o.position
    with pytest.raises(MucaError) as e:
        Solver(L, W, seed + 1).restore(state)
    assert e.value.code == _abi.MUCA_ERR_INVALID_ARG
    with pytest.raises(MucaError) as e:
        b.restore(state[:-4])
    assert e.value.code == _abi.MUCA_ERR_INVALID_ARG
