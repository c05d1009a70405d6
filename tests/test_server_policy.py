"""The serving queue's admission order and work estimate (host logic of the
server, csrc/muca_host_math.cpp), built alone with AddressSanitizer and
UndefinedBehaviourSanitizer and driven from here.  No device is involved.

* FIFO takes the oldest request;
* smallest-first takes the request of least estimated work, ties to the
  earlier arrival;
* a request queued longer than the wait bound goes first, the oldest such
  one first, so that a large request is not starved by a steady stream of
  small ones (checked by simulating the queue);
* the work estimate is walkers * N * sweeps with N/20 weight iterations
  (capped by max_iterations), checked on values worked by hand.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
CSRC = os.path.join(ROOT, "paper_1707_00919_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstring>
#include <vector>

#include "muca_host_math.h"

int main() {
    char op[16];
    while (scanf("%15s", op) == 1) {
        if (!strcmp(op, "pick")) {
            int sf; double now, wait; size_t n;
            if (scanf("%d %lf %lf %zu", &sf, &now, &wait, &n) != 4) return 2;
            std::vector<muca_host::QueuedJob> q(n);
            for (size_t i = 0; i < n; ++i)
                if (scanf("%lf %lf", &q[i].work, &q[i].t_submit) != 2) return 3;
            printf("%zu\n", muca_host::admission_pick(q.data(), n, sf != 0, now, wait));
        } else if (!strcmp(op, "work")) {
            unsigned L, W, it, is, mi, pt, ps;
            if (scanf("%u %u %u %u %u %u %u", &L, &W, &it, &is, &mi, &pt, &ps) != 7) return 4;
            printf("%.17g\n", muca_host::solve_work_estimate(L, W, it, is, mi, pt, ps));
        } else {
            return 5;
        }
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.fail("g++ is needed for the host-logic tests")
    d = tmp_path_factory.mktemp("policy")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + CSRC, str(src), os.path.join(CSRC, "muca_host_math.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)

    def run(lines):
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
        r = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True, text=True,
                           env=env, timeout=60)
        assert r.returncode == 0, r.stderr
        return r.stdout.split()

    return run


def pick(run, smallest_first, now, wait, jobs):
    line = "pick %d %r %r %d %s" % (smallest_first, now, wait, len(jobs),
                                    " ".join("%r %r" % j for j in jobs))
    return int(run([line])[0])


def test_fifo_takes_the_oldest(driver):
    jobs = [(5e9, 0.0), (1e6, 1.0), (1e3, 2.0)]
    assert pick(driver, 0, 100.0, 1.0, jobs) == 0


def test_smallest_first_takes_least_work_ties_to_earlier(driver):
    jobs = [(5e9, 0.0), (1e6, 1.0), (1e3, 2.0), (1e3, 3.0), (7e7, 4.0)]
    assert pick(driver, 1, 4.5, 30.0, jobs) == 2
    assert pick(driver, 1, 4.5, 30.0, [(2.0, 0.0), (2.0, 0.1), (3.0, 0.2)]) == 0


def test_overdue_request_goes_first_oldest_first(driver):
    jobs = [(1e3, 9.0), (5e9, 1.0), (7e9, 0.5), (1e2, 9.5)]
    # at t = 10 with a 5 s bound the requests of t = 1.0 and t = 0.5 are
    # overdue; the queue is in arrival order as the server keeps it, so the
    # first overdue entry is taken
    assert pick(driver, 1, 10.0, 5.0, jobs) == 1
    # nothing overdue: least work
    assert pick(driver, 1, 5.0, 5.0, jobs[1:3] + [(1e2, 4.9)]) == 2


def test_large_request_is_not_starved(driver):
    # one large request at t = 0, then a small one every 0.1 s; one request is
    # admitted every 0.1 s (the rest wait).  Without the bound the large one
    # would wait forever; with a 2 s bound it is admitted at the first
    # decision after it has waited 2 s.
    queue = [(1e12, 0.0)]
    admitted_big = None
    t = 0.0
    for step in range(1, 200):
        t = round(0.1 * step, 10)
        queue.append((1e6, t))           # arrival
        # queue entries stay in arrival order
        i = pick(driver, 1, t, 2.0, queue)
        job = queue.pop(i)
        if job[0] == 1e12:
            admitted_big = t
            break
        assert job[0] == 1e6
    assert admitted_big is not None and 2.0 < admitted_big <= 2.1 + 1e-9


def test_work_estimate_worked_by_hand(driver):
    out = driver(["work 32 16384 0 200 0 10000 10000",
                  "work 32 16384 0 200 10 10000 10000",
                  "work 8 100 5 20 0 30 50",
                  "work 4 64 0 2000 0 0 20000"])
    # L = 32: N = 1024, N/20 = 51.2 iterations of 200 sweeps = 10240, plus
    # 20000 production sweeps = 30240 sweeps; 16384 * 1024 * 30240
    assert float(out[0]) == 16384 * 1024 * 30240.0
    # capped at 10 iterations: 2000 + 20000 sweeps
    assert float(out[1]) == 16384 * 1024 * 22000.0
    # L = 8: N = 64, 3.2 iterations of 25 sweeps = 80, plus 80: 160 sweeps
    assert abs(float(out[2]) - 100 * 64 * 160.0) <= 1e-6
    # L = 4: N/20 = 0.8, at least one iteration: 2000 + 20000 sweeps
    assert float(out[3]) == 64 * 16 * 22000.0
