"""The serving form: every request's result is the same alone and in the mix.

Requests of mixed L and walker counts are submitted in two waves to a server
whose memory cap admits only a few at a time, so requests queue, join running
lanes and leave them while others run.  Each result (ln g bit for bit, the
iteration count, the status, the attempts) must equal that of the same solve
run alone through Solver, and that of the same solve run by the CPU oracle
(weight iterations to the flatness bound, Sec. 2.2 and Eq. 4; the production
run at the final weights and ln g, Sec. 3.3).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

REQUESTS = [(8, 100, 1), (8, 300, 2), (12, 64, 3), (16, 200, 4), (12, 130, 5), (8, 65, 6),
            (16, 70, 7), (10, 90, 8)]
KW = dict(iter_sweeps=20, min_flatness=0.3, max_iterations=40, prod_therm=30, prod_sweeps=50)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    yield


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def solo(L, W, seed):
    from paper_1707_00919_amd import MucaError, Solver
    s = Solver(L, W, seed, use_torch=False)
    it = 0
    flat = False
    while it < KW["max_iterations"]:
        info = s.iterate(0, KW["iter_sweeps"])
        it += 1
        if info["flatness"] >= KW["min_flatness"]:
            flat = True
            break
    s.production(KW["prod_therm"], KW["prod_sweeps"])
    try:
        lng = s.log_dos(0)
    except MucaError:
        lng = np.zeros(L * L + 1)
    s.close()
    return it, flat, lng


def oracle_solve(L, W, seed):
    """The request's solve on the CPU oracle: the server's schedule (weight
    iterations until the flatness bound or the iteration cap, then the
    production run in one call) and ln g with ln g(E_min) = ln 2."""
    import oracle
    o = oracle.OracleMuca(L, W, seed)
    it = 0
    flat = False
    while it < KW["max_iterations"]:
        info = o.iterate(0, KW["iter_sweeps"])
        it += 1
        if info["flatness"] >= KW["min_flatness"]:
            flat = True
            break
    o.production(KW["prod_therm"], KW["prod_sweeps"])
    lng = o.log_dos(0)
    return it, flat, (np.zeros(L * L + 1) if lng is None else lng)


@pytest.mark.parametrize("batch_flags,policy", [(0, "fifo"), (3, "fifo"), (3, "smallest-first")])
def test_served_equals_alone(batch_flags, policy):
    from paper_1707_00919_amd import Server, state_bytes
    note("server mix, batch_flags=%d, policy=%s" % (batch_flags, policy))
    cap = sum(sorted(state_bytes(L, W) for L, W, _ in REQUESTS)[-3:]) + 4096
    srv = Server(cap, batch_flags=batch_flags, policy=policy)
    tickets = [srv.submit(L, W, s, **KW) for L, W, s in REQUESTS[:5]]
    max_resident = 0
    saw_queue = False
    for _ in range(20):
        srv.progress()
        st = srv.stats()
        max_resident = max(max_resident, st["resident_bytes"])
        saw_queue |= st["queued"] > 0
    tickets += [srv.submit(L, W, s, **KW) for L, W, s in REQUESTS[5:]]
    st = srv.stats()
    saw_queue |= st["queued"] > 0
    out = srv.drain(tickets, timeout_s=120.0)
    st = srv.stats()
    assert st["completed"] == len(REQUESTS) and st["active"] == 0 and st["queued"] == 0
    assert st["resident_bytes"] == 0
    assert saw_queue and max_resident <= cap
    # continuous batching, not a queue: requests of different L were resident
    # at the same time, and a request admitted only after another had finished
    # (it waited for room) joined while a third, admitted before it, still ran
    res = [out[t][0] for t in tickets]
    overlap = lambda a, b: res[a]["t_admit"] < res[b]["t_done"] and res[b]["t_admit"] < res[a]["t_done"]
    n = len(REQUESTS)
    assert any(overlap(i, j) and REQUESTS[i][0] != REQUESTS[j][0] for i in range(n) for j in range(i + 1, n))
    first_done = min(r["t_done"] for r in res)
    assert any(res[j]["t_admit"] >= first_done and res[i]["t_admit"] < res[j]["t_admit"] < res[i]["t_done"]
               for i in range(n) for j in range(n) if i != j)
    for t, (L, W, seed) in zip(tickets, REQUESTS):
        res, lng = out[t]
        it, flat, ref = solo(L, W, seed)
        assert res["iterations"] == it
        assert res["status"] == (0 if flat else 5)
        assert res["attempts"] == W * L * L * (KW["iter_sweeps"] * it + KW["prod_therm"] + KW["prod_sweeps"])
        assert res["t_submit"] <= res["t_admit"] <= res["t_weights"] <= res["t_done"]
        np.testing.assert_array_equal(lng.view(np.uint64), ref.view(np.uint64))
        # the same request on the CPU oracle
        oit, oflat, oref = oracle_solve(L, W, seed)
        assert res["iterations"] == oit
        assert res["status"] == (0 if oflat else 5)
        np.testing.assert_array_equal(lng.view(np.uint64), oref.view(np.uint64))
    srv.close()


def test_server_rejects_bad_requests():
    from paper_1707_00919_amd import MucaError, Server, _abi, state_bytes
    note("server errors")
    srv = Server(state_bytes(8, 64) + 4096)
    with pytest.raises(MucaError) as e:
        srv.submit(7, 64, 1)
    assert e.value.code == _abi.MUCA_ERR_INVALID_ARG
    with pytest.raises(MucaError):
        srv.submit(8, 64, 1, iter_sweeps=0)
    big = srv.submit(32, 4096, 1, **KW)      # larger than the whole cap
    ok = srv.submit(8, 64, 2, **KW)
    out = srv.drain([big, ok], timeout_s=60.0)
    assert out[big][0]["status"] == _abi.MUCA_ERR_OUT_OF_MEMORY
    assert out[ok][0]["status"] in (0, 5)
    srv.close()


def test_smallest_first_admission_order():
    # one request resident at a time (walker budget 1): smallest-first admits
    # in order of estimated work, FIFO in arrival order; results are the same
    from paper_1707_00919_amd import Server
    note("server admission order")
    reqs = [(16, 512, 11), (8, 64, 12), (12, 100, 13), (8, 80, 14)]
    kw = dict(KW, max_iterations=3)
    order = {}
    lngs = {}
    for policy in ("fifo", "smallest-first"):
        srv = Server(1 << 30, max_active_walkers=1, policy=policy)
        tickets = [srv.submit(L, W, s, **kw) for L, W, s in reqs]
        out = srv.drain(tickets, timeout_s=120.0)
        t_admit = [out[t][0]["t_admit"] for t in tickets]
        order[policy] = sorted(range(len(reqs)), key=lambda i: t_admit[i])
        lngs[policy] = [out[t][1] for t in tickets]
        srv.close()
    assert order["fifo"] == [0, 1, 2, 3]
    assert order["smallest-first"] == [1, 3, 2, 0]
    for a, b in zip(lngs["fifo"], lngs["smallest-first"]):
        np.testing.assert_array_equal(a.view(np.uint64), b.view(np.uint64))


def test_smallest_first_wait_is_bounded():
    # a large request queued behind a steady stream of small ones is admitted
    # once it has waited max_wait_s: no small request is admitted after that
    # while it waits (slack: one small solve and the admission step)
    import time
    from paper_1707_00919_amd import Server
    note("server wait bound")
    max_wait = 0.5
    small = dict(iter_sweeps=5, min_flatness=1.0, max_iterations=2, prod_therm=0, prod_sweeps=5)
    srv = Server(1 << 30, max_active_walkers=1, policy="smallest-first", max_wait_s=max_wait)
    first = srv.submit(8, 64, 100, **small)     # occupies the device first
    srv.progress()
    big = srv.submit(16, 1024, 101, **small)
    smalls = [first]
    t0 = time.monotonic()
    seed = 200
    while time.monotonic() - t0 < 3.0:
        if srv.stats()["queued"] < 4:
            smalls.append(srv.submit(8, 64, seed, **small))
            seed += 1
        if not srv.progress():
            time.sleep(2e-4)
    out = srv.drain(smalls + [big], timeout_s=120.0)
    srv.close()
    rb = out[big][0]
    assert rb["status"] in (0, 5)
    before = [out[t][0] for t in smalls if out[t][0]["t_admit"] < rb["t_admit"]]
    assert len(before) >= 2, "smallest-first let the large request go first"
    # every small admitted before the large one was admitted by the time the
    # large one had waited max_wait_s plus one small solve
    slack = max(r["t_done"] - r["t_admit"] for r in before) + 0.05
    assert all(r["t_admit"] <= rb["t_submit"] + max_wait + slack for r in before)
    assert rb["t_admit"] - rb["t_submit"] <= max_wait + slack + 0.5
