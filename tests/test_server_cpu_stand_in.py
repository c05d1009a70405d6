"""The serving form's host code on a CPU stand-in for HIP, under the sanitizers.

libmuca's host sources (muca_runtime.cpp, muca_batch.cpp, muca_server.cpp,
muca_host_math.cpp) are built with g++ against tests/cpu_hip/: a stand-in for
the HIP calls they make (streams as worker threads, events, stream capture into
graphs with host nodes, allocations checked by range and kind) and for the
kernels (each checks its arguments as the real kernel uses them and adds the
histogram counts the host expects; a flat histogram takes about log2(N / 16)
weight iterations).  tests/cpu_hip/served_stream.cpp then runs the served
workload's own request stream (muca_inputs.serving_requests: Poisson arrivals,
L in {16, 24, 32, 48, 64}, 1024-16384 walkers) through the server, time-scaled,
and checks every result (status, iterations, attempts, ln g finite) and, for a
sample, that ln g is bit-identical to the same request solved alone.
tests/cpu_hip/launch_order.cpp checks the order and staggering of a batched
round's launches on the same stand-in.

Frees do not wait for queued work here (CPU_HIP_FREE_NOWAIT=1), so that work
still queued on freed memory would trip AddressSanitizer or the range checks.
No device is involved.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
CSRC = os.path.join(ROOT, "paper_1707_00919_amd", "csrc")
STAND_IN = os.path.join(ROOT, "tests", "cpu_hip")
LIBRARY = [os.path.join(CSRC, f) for f in ("muca_runtime.cpp", "muca_batch.cpp", "muca_server.cpp",
                                           "muca_host_math.cpp")] + [os.path.join(STAND_IN, "cpu_hip.cpp")]

FIFO, SMALLEST_FIRST = 0, 1
GRAPH, AUTOTUNE = 1, 2


def _build(tmp, name, sanitize, driver="served_stream.cpp"):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = os.path.join(str(tmp), name)
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + sanitize,
           "-Wno-attributes", "-pthread", "-I" + STAND_IN, "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    if sanitize != "thread":
        cmd.append("-fno-sanitize-recover=all")
    sources = LIBRARY + [os.path.join(STAND_IN, driver)]
    r = subprocess.run(cmd + sources + ["-o", exe, "-lm"], capture_output=True, text=True)
    if r.returncode != 0 and "san" in (r.stderr or "").lower() and "cannot find" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _write(d, name, reqs):
    p = d / name
    p.write_text("".join("%.9f %d %d %d\n" % r for r in reqs))
    return str(p), len(reqs)


@pytest.fixture(scope="module")
def streams(tmp_path_factory):
    """The whole served stream (1203 requests over 60 s) and its first 20 s."""
    sys.path.insert(0, ROOT)
    from muca_inputs import serving_requests
    reqs = serving_requests()
    d = tmp_path_factory.mktemp("served")
    return {"whole": _write(d, "whole.txt", reqs), "head": _write(d, "head.txt", [r for r in reqs if r[0] < 20.0])}


@pytest.fixture(scope="module")
def asan(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("served_asan"), "served_asan", "address,undefined")


@pytest.fixture(scope="module")
def tsan(tmp_path_factory):
    return _build(tmp_path_factory.mktemp("served_tsan"), "served_tsan", "thread")


def _run(exe, stream, flags, policy, scale=20.0, solo_every=100, env=None, timeout=600):
    path, n = stream
    e = dict(os.environ, CPU_HIP_FREE_NOWAIT="1", CPU_HIP_RATE="8e12")
    e.update(env or {})
    # the whole workload's memory cap and walker budget of the served benchmark
    args = [exe, path, str(64 << 30), str(1 << 19), str(flags), str(policy), str(scale), str(solo_every)]
    r = subprocess.run(args, capture_output=True, text=True, timeout=timeout, env=e)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    words = r.stdout.strip().splitlines()[-1].split()
    assert words[:2] == ["ok", str(n)], out[-2000:]
    assert int(words[3]) > 0  # some requests were compared with their solo solves
    return words


def test_whole_served_stream_under_asan(asan, streams):
    """The served benchmark's configuration: graph rounds, arrival order."""
    _run(asan, streams["whole"], GRAPH, FIFO)


@pytest.mark.parametrize("flags,policy", [(GRAPH, SMALLEST_FIRST), (0, FIFO), (GRAPH | AUTOTUNE, FIFO)],
                         ids=["graph-smallest-first", "no-graph-fifo", "graph-autotune-fifo"])
def test_served_stream_head_under_asan(asan, streams, flags, policy):
    _run(asan, streams["head"], flags, policy)


def test_served_stream_head_under_tsan(tsan, streams):
    """Graph rounds end in a host node on a stream worker thread while the
    driver thread admits, launches and collects other lanes."""
    _run(tsan, streams["head"], GRAPH, FIFO, solo_every=50, env={"TSAN_OPTIONS": "halt_on_error=1"})


def test_batched_launch_order(tmp_path):
    """A batched round issues its two-wave launches first, each kind by its
    longest chain, and staggers the starts (30 us more per launch) in crowded
    and paired rounds only; with and without the captured graph
    (tests/cpu_hip/launch_order.cpp)."""
    exe = _build(tmp_path, "launch_order", "address,undefined", driver="launch_order.cpp")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=dict(os.environ, CPU_HIP_RATE="0"))
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert r.stdout.strip().splitlines()[-1] == "ok"
