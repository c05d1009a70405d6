"""The batched form against single-instance runs and the oracle.

A batch sweeps many independent instances (mixed L and walker counts) in
shared launches; every member's histogram, weights, spins and energies must
equal, bit for bit, those of the same instance run alone -- with and without
HIP-graph replay, with the kernel-form autotuner, and when members need more
than one launch per round.
"""
import sys

import numpy as np
import pytest

import oracle
from muca_inputs import random_log_weights, smooth_log_weights

pytestmark = pytest.mark.gpu

SHAPES = [(8, 300, 1), (12, 64, 2), (16, 1000, 3), (24, 130, 4), (32, 700, 5), (48, 100, 6),
          (62, 70, 7), (64, 128, 8), (96, 65, 9), (6, 65, 10)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    yield


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def make(shapes, flags=0):
    from paper_1707_00919_amd import Solver
    out = []
    for L, W, seed in shapes:
        s = Solver(L, W, seed, flags=flags)
        s.set_log_weights(smooth_log_weights(L, seed))
        out.append(s)
    return out


def same(a, b):
    np.testing.assert_array_equal(a.histogram(), b.histogram())
    np.testing.assert_array_equal(bits(a.log_weights()), bits(b.log_weights()))
    np.testing.assert_array_equal(a.energies(), b.energies())
    np.testing.assert_array_equal(a.spins(), b.spins())


# rounds: (modes, therm, sweeps) per member
ROUNDS = [
    ([1] * 10, [1] * 10, [2] * 10),
    ([1, 2, 1, 0, 1, 2, 1, 1, 2, 1], [0, 2, 1, 0, 0, 1, 1, 0, 0, 3], [3, 2, 1, 0, 2, 3, 2, 1, 2, 2]),
    ([2] * 10, [0] * 10, [2] * 10),
]


@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_batch_matches_solo(flags):
    from paper_1707_00919_amd import Batch
    note("batch vs solo flags=%d" % flags)
    solo = make(SHAPES)
    grouped = make(SHAPES)
    batch = Batch(grouped, flags=flags)
    wide = SHAPES.index((96, 65, 9))
    wide_forms = set()
    for modes, therm, sweeps in ROUNDS + ROUNDS[:1]:
        infos = batch.run(modes, therm, sweeps)
        wide_forms.add(infos[wide]["kernel_variant"])
        for i, s in enumerate(solo):
            if modes[i] == 1:
                si = s.iterate(therm[i], sweeps[i])
            elif modes[i] == 2:
                si = s.production(therm[i], sweeps[i])
            else:
                continue
            assert infos[i]["hist_sum"] == si["hist_sum"]
            assert infos[i]["flatness"] == si["flatness"]
            assert infos[i]["sweep_counter"] == si["sweep_counter"]
    for a, b in zip(solo, grouped):
        same(a, b)
    # every round's two-wave workgroups fit on the device at once, so every
    # round runs the two-wave form, with the autotuner too: the L = 96 member
    # ran the two-wave wide form only
    assert wide_forms == {4}
    batch.close()


# a batch whose two-wave workgroups do not all fit, not even with two chains
# per CU: L = 64 and L = 48 members of 257 blocks each (one two-wave
# workgroup per CU, or one pair) beside small members
CROWDED = [(64, 16448, 21), (48, 16448, 26), (8, 300, 22), (16, 1000, 23), (96, 65, 24), (32, 130, 25)]
CROWDED_ROUNDS = [
    ([1] * 6, [0] * 6, [1] * 6),
    ([2, 1, 1, 2, 1, 2], [1, 0, 1, 0, 1, 0], [1, 2, 2, 1, 1, 2]),
    ([1, 2, 2, 0, 2, 1], [0, 1, 0, 0, 0, 1], [2, 1, 1, 0, 2, 1]),
    ([2] * 6, [0] * 6, [1] * 6),
    ([1] * 6, [1] * 6, [1] * 6),
    ([2] * 6, [0] * 6, [2] * 6),
]


@pytest.mark.parametrize("flags", [0, 2])
def test_crowded_batch_mixed_and_one_wave_shapes_match_solo(flags):
    # without the autotuner every round runs the mixed-longest shape: the
    # two-wave form only for the longest chain (L = 96), the one-wave form for
    # the rest; with it the first five rounds time the mixed-longest shape, the
    # mixed shape (the longest chains first in the two-wave form while they
    # fit: L = 96, then L = 64 in pairs), both one-wave shapes and the
    # split-merge cadence, and later rounds keep the fastest; every member
    # stays bit for bit equal to its solo run
    from paper_1707_00919_amd import Batch
    note("crowded batch flags=%d" % flags)
    solo = make(CROWDED)
    grouped = make(CROWDED)
    batch = Batch(grouped, flags=flags)
    forms = [set() for _ in CROWDED]
    for modes, therm, sweeps in CROWDED_ROUNDS:
        infos = batch.run(modes, therm, sweeps)
        for i, s in enumerate(solo):
            if modes[i] == 1:
                si = s.iterate(therm[i], sweeps[i])
            elif modes[i] == 2:
                si = s.production(therm[i], sweeps[i])
            else:
                continue
            forms[i].add(infos[i]["kernel_variant"])
            assert infos[i]["hist_sum"] == si["hist_sum"]
            assert infos[i]["flatness"] == si["flatness"]
            assert infos[i]["sweep_counter"] == si["sweep_counter"]
    for a, b in zip(solo, grouped):
        same(a, b)
    assert forms[1] == forms[2] == forms[3] == forms[5] == {1}  # one-wave in every shape
    if flags & 2:
        assert forms[0] == {1, 5} and forms[4] == {3, 4}
    else:
        assert forms[0] == {1} and forms[4] == {4}
    batch.close()


def test_batch_matches_oracle_and_splits_launches():
    # a member capped at 2 sweeps per launch forces several launch chunks
    from paper_1707_00919_amd import Batch, Solver
    note("batch vs oracle, chunked")
    shapes = [(8, 70, 11), (16, 64, 12), (20, 65, 13)]
    members = [Solver(L, W, s, flags=2 if i == 1 else 0) for i, (L, W, s) in enumerate(shapes)]
    orcs = [oracle.OracleMuca(L, W, s) for L, W, s in shapes]
    for (L, W, s), m, o in zip(shapes, members, orcs):
        om = random_log_weights(L, s, scale=2.0)
        m.set_log_weights(om)
        o.set_log_weights(om)
    batch = Batch(members)
    infos = batch.run([1, 1, 2], [1, 2, 0], [3, 5, 2])
    for (m, o, th, sw, md) in zip(members, orcs, [1, 2, 0], [3, 5, 2], [1, 1, 2]):
        (o.iterate if md == 1 else o.production)(th, sw)
        np.testing.assert_array_equal(m.histogram(), o.hist)
        np.testing.assert_array_equal(bits(m.log_weights()), bits(o.omega))
        np.testing.assert_array_equal(m.energies(), o.energies)
        np.testing.assert_array_equal(m.spins(), o.spins)
    assert infos[1]["kernel_launches"] >= 3
    batch.close()


def test_graph_replays_match_eager_rounds():
    # the same round shape replayed from one captured graph, with eager work
    # and synchronisations in between, against an eager batch
    from paper_1707_00919_amd import Batch, _abi
    note("graph replays")
    shapes = SHAPES[:5]
    eager = make(shapes)
    graphed = make(shapes)
    be = Batch(eager)
    bg = Batch(graphed, flags=_abi.MUCA_BATCH_GRAPH)
    for r in range(4):
        be.run([1] * 5, [0] * 5, [2] * 5)
        bg.run([1] * 5, [0] * 5, [2] * 5)
        for a, b in zip(eager, graphed):
            np.testing.assert_array_equal(a.histogram(), b.histogram())
            np.testing.assert_array_equal(bits(a.log_weights()), bits(b.log_weights()))
    for a, b in zip(eager, graphed):
        same(a, b)


def test_batch_rejects_bad_arguments():
    from paper_1707_00919_amd import Batch, MucaError, _abi
    note("batch errors")
    members = make(SHAPES[:2])
    with pytest.raises(MucaError) as e:
        Batch([members[0], members[0]])
    assert e.value.code == _abi.MUCA_ERR_INVALID_ARG
    b = Batch(members)
    with pytest.raises(MucaError) as e:
        b.run([3, 1], [0, 0], [1, 1])
    assert e.value.code == _abi.MUCA_ERR_INVALID_ARG
    b.run([0, 0], [0, 0], [1, 1])   # nothing to do


def test_two_batches_in_flight():
    # two batches submitted back to back run side by side; each member still
    # matches its solo run, and out-of-order calls are refused
    import time
    from paper_1707_00919_amd import Batch, MucaError, _abi
    note("two batches in flight")
    shapes_a, shapes_b = SHAPES[:4], SHAPES[4:8]
    solo = make(shapes_a + shapes_b)
    ma, mb = make(shapes_a), make(shapes_b)
    ba, bb = Batch(ma, use_torch=False), Batch(mb, use_torch=False)
    with pytest.raises(MucaError) as e:
        ba.finish()
    assert e.value.code == _abi.MUCA_ERR_STATE
    for r in range(3):
        ba.submit([1] * 4, [1] * 4, [3] * 4)
        bb.submit([2] * 4, [0] * 4, [4] * 4)
        with pytest.raises(MucaError) as e:
            ba.submit([1] * 4, [1] * 4, [3] * 4)
        assert e.value.code == _abi.MUCA_ERR_STATE
        t0 = time.time()
        while not (ba.done() and bb.done()):
            assert time.time() - t0 < 60.0
            time.sleep(0.001)
        ia, ib = ba.finish(), bb.finish()
        assert all(i["sweep_counter"] == 4 * (r + 1) for i in ia + ib)
        for s in solo[:4]:
            s.iterate(1, 3)
        for s in solo[4:]:
            s.production(0, 4)
    for a, b in zip(solo, ma + mb):
        same(a, b)


def test_changing_membership():
    # members join and leave between rounds (continuous batching); buffers are
    # reused or grown, and every instance still matches its solo run
    from paper_1707_00919_amd import Batch, _abi
    note("changing membership")
    solo = make(SHAPES)
    pool = make(SHAPES)
    b = Batch(pool[:2], flags=_abi.MUCA_BATCH_GRAPH)
    plan = [[0, 1], [0, 1, 2], [2, 3], [3, 4, 5, 6, 7, 8, 9], [0, 9], [5]]
    for r, idx in enumerate(plan):
        b.set_members([pool[i] for i in idx])
        n = len(idx)
        infos = b.run([1] * n, [r % 2] * n, [2] * n)
        for k, i in enumerate(idx):
            si = solo[i].iterate(r % 2, 2)
            assert infos[k]["sweep_counter"] == si["sweep_counter"]
    for a, c in zip(solo, pool):
        same(a, c)


def test_batched_workload_full_size_sampled_walkers():
    # the 48 instances of the batched workload at their full sizes, in the
    # launch form the benchmark uses (graph + autotune, two rounds so that
    # both kernel forms run): sampled walkers of every instance against the
    # oracle run on just those walkers
    from paper_1707_00919_amd import Batch, Solver, _abi
    from muca_inputs import batch_instances
    note("batched workload, full size, sampled walkers")
    inst = batch_instances()
    members = [Solver(L, W, sd) for L, W, sd in inst]
    oms = [smooth_log_weights(L, sd + 7) for L, _, sd in inst]
    for m, om in zip(members, oms):
        m.set_log_weights(om)
    b = Batch(members, flags=_abi.MUCA_BATCH_GRAPH | _abi.MUCA_BATCH_AUTOTUNE)
    forms = set()
    for _ in range(2):
        infos = b.run([2] * len(members), 1, 1)
        forms |= {i["kernel_variant"] for i in infos}
    # a one-wave and a two-wave form (single or in pairs) both ran
    assert 1 in forms and forms & {2, 5} and forms <= {1, 2, 5}
    rng = np.random.default_rng(5)
    for (L, W, sd), m, om in zip(inst, members, oms):
        ids = np.unique(np.concatenate([[0, W - 1], rng.integers(0, W, 6)])).astype(np.uint32)
        o = oracle.OracleMuca(L, W, sd, walker_ids=ids)
        o.set_log_weights(om)
        o.production(1, 1)
        o.production(1, 1)
        np.testing.assert_array_equal(m.energies()[ids], o.energies)
        np.testing.assert_array_equal(m.spins()[ids], o.spins)


def test_batched_workload_full_size_iterations_match_oracle():
    # the 48 instances at their full sizes in the benchmark's launch form
    # (graph + autotune: the first round runs the mixed-longest shape, the
    # L = 64 members in pairs, the second the mixed shape, the L = 48 and
    # L = 64 members in pairs), two weight
    # iterations of one unrecorded and one recorded sweep; every member's
    # histogram and omega bit patterns, and every walker's spins and energy,
    # against the oracle run on all walkers
    from paper_1707_00919_amd import Batch, Solver, _abi
    from muca_inputs import batch_instances
    note("batched workload, full size, all walkers, two iterations")
    inst = batch_instances()
    members = [Solver(L, W, sd) for L, W, sd in inst]
    oms = [smooth_log_weights(L, sd + 11) for L, _, sd in inst]
    for m, om in zip(members, oms):
        m.set_log_weights(om)
    b = Batch(members, flags=_abi.MUCA_BATCH_GRAPH | _abi.MUCA_BATCH_AUTOTUNE)
    hists, forms = [[] for _ in inst], set()
    for _ in range(2):
        infos = b.run([1] * len(members), 1, 1)
        forms |= {i["kernel_variant"] for i in infos}
        for k, m in enumerate(members):
            hists[k].append(m.histogram())
    assert 1 in forms and forms & {2, 5}
    for k, ((L, W, sd), m, om) in enumerate(zip(inst, members, oms)):
        o = oracle.OracleMuca(L, W, sd)
        o.set_log_weights(om)
        for r in range(2):
            o.iterate(1, 1)
            np.testing.assert_array_equal(hists[k][r], o.hist)
        np.testing.assert_array_equal(bits(m.log_weights()), bits(o.omega))
        np.testing.assert_array_equal(m.energies(), o.energies)
        np.testing.assert_array_equal(m.spins(), o.spins)
    b.close()


def test_batch_member_with_zero_threshold_runs_generic():
    # a member whose table has a reachable T = 0 runs the generic kernel in
    # its own group, next to members on the other forms; all match their
    # solo runs
    from paper_1707_00919_amd import Batch
    note("batch with a zero-threshold member")
    shapes = [(8, 64, 51), (16, 130, 52), (96, 64, 53)]
    oms = [random_log_weights(L, s, scale=1.0) for L, _, s in shapes]
    oms[0] = oms[0].copy()
    oms[0][30:] -= 30.0
    solo, grouped = make(shapes), make(shapes)
    for a, b, om in zip(solo, grouped, oms):
        a.set_log_weights(om)
        b.set_log_weights(om)
    batch = Batch(grouped)
    infos = batch.run([2, 1, 1], [1, 0, 1], [2, 3, 2])
    assert infos[0]["kernel_variant"] == 0 and infos[2]["kernel_variant"] == 4  # L = 96: wide, two waves
    solo[0].production(1, 2)
    solo[1].iterate(0, 3)
    solo[2].iterate(1, 2)
    for a, b in zip(solo, grouped):
        same(a, b)


def test_batched_solves_with_sliced_production_match_oracle():
    # the benchmark's batched solve (bench.batched_solve): weight iterations to
    # the flatness bound, then the production run in slices from the round
    # after each member's last iteration, ln g from the summed slices -- each
    # member's iteration count and ln g bits equal the oracle's single solve
    # (Sec. 2.2 and Eq. 4; Sec. 3.3)
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    from paper_1707_00919_amd import Batch, Solver, _abi
    inst = [(8, 64, 21), (12, 100, 22), (16, 70, 23), (8, 200, 24)]
    it_sw, flat, max_it, p_th, p_sw = 20, 0.3, 25, 30, 50
    note("batched solves with sliced production vs oracle")
    att, iters, lngs, rounds, _ = bench.batched_solve(
        Batch, Solver, inst, _abi.MUCA_BATCH_GRAPH, it_sw, flat, max_it, p_th, p_sw)
    for (L, W, seed), it, lng in zip(inst, iters, lngs):
        o = oracle.OracleMuca(L, W, seed)
        oit = 0
        while oit < max_it:
            info = o.iterate(0, it_sw)
            oit += 1
            if info["flatness"] >= flat:
                break
        o.production(p_th, p_sw)
        ref = o.log_dos(0)
        assert it == oit, (L, W, seed)
        ref = np.zeros(L * L + 1) if ref is None else ref
        np.testing.assert_array_equal(bits(lng), bits(ref))
    # production slices of at most it_sw sweeps: at least (p_th + p_sw) / it_sw
    # rounds after the last member's last iteration
    assert rounds >= max(iters) + (p_th + p_sw + it_sw - 1) // it_sw
    assert att == sum(W * L * L * (it_sw * it + p_th + p_sw) for (L, W, _), it in zip(inst, iters))
