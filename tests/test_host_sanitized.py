"""The library's host arithmetic built alone with AddressSanitizer and
UndefinedBehaviourSanitizer and run on seeded inputs, with its results checked
against the oracle or against definitions.  No device is involved: these
sources include no HIP.

* csrc/muca_host_math.cpp: thresholds and their kernel encodings, flatness,
  Chebyshev distance, KL divergence, covered ranges and ln g (against the
  oracle); the cut of a call into sweep segments (attempt by attempt it must
  cover exactly the attempts of the call, in order, and attempt p is recorded
  iff p >= pos0 + therm); the serving form's arena (offset for offset the same
  as first fit with coalescing written out from its definition, live ranges
  disjoint and inside the arena).
* csrc/muca_analysis.cpp: jackknife and canonical reweighting (against the
  oracle)."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
import oracle.analysis as oan
from muca_inputs import random_log_weights, smooth_log_weights

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
CSRC = os.path.join(ROOT, "paper_1707_00919_amd", "csrc")

DRIVER = r"""
#include <cstdint>
#include <cstdio>
#include <vector>

#include "muca.h"
#include "muca_host_math.h"

template <class T> static void rd(std::vector<T>& v, size_t n) {
    v.resize(n);
    if (n && fread(v.data(), sizeof(T), n, stdin) != n) throw 1;
}
template <class T> static void wr(const T* p, size_t n) { fwrite(p, sizeof(T), n, stdout); }
template <class T> static void wr1(T x) { fwrite(&x, sizeof(T), 1, stdout); }

int main() {
    uint32_t hdr[5];
    if (fread(hdr, 4, 5, stdin) != 5) return 2;
    const uint32_t L = hdr[0], blocks = hdr[1], nbeta = hdr[2], ncut = hdr[3];
    const int reach_prev = (int)hdr[4];
    const uint32_t N = L * L;
    std::vector<double> om, betas;
    std::vector<uint64_t> H, bh, cuts;
    rd(om, N + 1); rd(H, N + 1); rd(bh, (size_t)blocks * (N + 1)); rd(betas, nbeta); rd(cuts, 3 * (size_t)ncut);

    std::vector<uint64_t> t5((size_t)(N + 1) * 5), t4((size_t)(N + 1) * 4);
    std::vector<uint32_t> f5((size_t)(N + 1) * 5), f8((size_t)(N + 1) * 8);
    muca_host::compute_thresholds(N, om.data(), t5.data());
    muca_host::device_table(N, t5.data(), t4.data());
    const uint32_t ok5 = muca_host::fast_table(N, t5.data(), f5.data(), 5);
    const uint32_t ok8 = muca_host::fast_table(N, t5.data(), f8.data(), 8);
    wr(t5.data(), t5.size()); wr(t4.data(), t4.size());
    wr1(ok5); wr(f5.data(), f5.size()); wr1(ok8); wr(f8.data(), f8.size());
    wr1(muca_host::flatness_of(N, H.data()));
    wr1(muca_host::chebyshev_of(N, H.data()));
    wr1(muca_host::kl_of(N, H.data(), reach_prev));
    wr1((int32_t)muca_host::reach_of(N, H.data()));
    wr1((int32_t)muca_host::width_of(N, H.data()));
    std::vector<double> lg(N + 1), err(N + 1);
    for (int norm = 0; norm < 2; ++norm) {
        wr1((int32_t)muca_host::log_dos_of(N, H.data(), om.data(), norm, lg.data()));
        wr(lg.data(), lg.size());
    }
    wr1((int32_t)muca_jackknife_log_dos(L, blocks, bh.data(), om.data(), 1, lg.data(), err.data()));
    wr(lg.data(), lg.size()); wr(err.data(), err.size());
    std::vector<double> e(nbeta), ee(nbeta), c(nbeta), ce(nbeta);
    wr1((int32_t)muca_canonical(L, blocks, bh.data(), om.data(), nbeta, betas.data(), e.data(), ee.data(),
                                c.data(), ce.data()));
    wr(e.data(), nbeta); wr(ee.data(), nbeta); wr(c.data(), nbeta); wr(ce.data(), nbeta);
    // arena: a sequence of allocations and releases (of earlier allocations)
    uint64_t arena_hdr[2];
    if (fread(arena_hdr, 8, 2, stdin) != 2) return 3;
    std::vector<uint64_t> ops;
    rd(ops, 2 * (size_t)arena_hdr[0]);
    muca_host::Arena arena;
    arena.reset(arena_hdr[1]);
    std::vector<uint64_t> offs, sizes;
    for (uint64_t i = 0; i < arena_hdr[0]; ++i) {
        if (ops[2 * i] == 0) {
            size_t off = 0;
            const bool ok = arena.alloc(ops[2 * i + 1], &off);
            offs.push_back(ok ? off : ~0ull);
            sizes.push_back(ops[2 * i + 1]);
            const uint64_t o[2] = {ok ? 1ull : 0ull, ok ? (uint64_t)off : 0ull};
            wr(o, 2);
        } else {
            const size_t j = ops[2 * i + 1];
            const bool held = offs[j] != ~0ull;  // releasing a failed allocation is a no-op
            if (held)
                arena.release(offs[j], sizes[j]);
            const uint64_t o[2] = {held ? 2ull : 3ull, 0ull};
            wr(o, 2);
        }
        wr1((uint64_t)arena.used());
    }
    for (uint32_t i = 0; i < ncut; ++i) {
        const auto segs = muca_host::segments_of(N, cuts[3 * i], cuts[3 * i + 1], cuts[3 * i + 2]);
        wr1((uint32_t)segs.size());
        for (const auto& g : segs) {
            const uint64_t a[3] = {g.sweep0, g.n, g.therm};
            const uint32_t b[3] = {g.site_begin, g.site_end, g.rec_begin};
            wr(a, 3); wr(b, 3);
        }
    }
    return 0;
}
"""

CUTS = [(0, 0, 16), (0, 16, 16), (3, 5, 40), (7, 0, 9), (16, 3, 0), (5, 30, 2), (0, 33, 31), (17, 15, 1)]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("host_asan")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "host_asan"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(CSRC, "muca_host_math.cpp"), os.path.join(CSRC, "muca_analysis.cpp"), str(src),
           "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    return str(exe)


class Reader:
    def __init__(self, buf):
        self.buf, self.at = buf, 0

    def take(self, dtype, n):
        a = np.frombuffer(self.buf, dtype=dtype, count=n, offset=self.at)
        self.at += a.nbytes
        return a

    def one(self, dtype):
        return self.take(dtype, 1)[0]


def arena_ops(seed, n=400):
    """A seeded mix of allocations (sizes 1 byte .. 40 KiB) and releases of
    earlier ones, as (kind, arg) pairs: kind 0 allocates arg bytes, kind 1
    releases allocation number arg (a no-op if that allocation failed)."""
    rng = np.random.default_rng(seed)
    ops, live, k = [], [], 0
    for _ in range(n):
        if live and rng.random() < 0.45:
            ops.append((1, live.pop(int(rng.integers(0, len(live))))))
        else:
            ops.append((0, int(rng.integers(1, 40 * 1024))))
            live.append(k)
            k += 1
    return ops


def model_arena(size, ops):
    """First fit with coalescing, written from its definition: sizes round
    up to 256 bytes; an allocation takes the start of the lowest-addressed
    free range that holds it; a release returns its range and merges it with
    free neighbours.  Returns per op (status, offset, bytes in use); status
    1 allocated, 0 no room, 2 released, 3 nothing to release."""
    free = [[0, size]] if size else []
    out, allocs, used = [], [], 0
    for kind, a in ops:
        if kind == 0:
            n = -(-a // 256) * 256
            hit = next((f for f in free if f[1] >= n), None)
            if hit is None:
                allocs.append(None)
                out.append((0, 0, used))
                continue
            off = hit[0]
            hit[0] += n
            hit[1] -= n
            free = [f for f in free if f[1] > 0]
            used += n
            allocs.append((off, n))
            out.append((1, off, used))
        else:
            if allocs[a] is None:  # that allocation failed: nothing to release
                out.append((3, 0, used))
                continue
            off, n = allocs[a]
            used -= n
            free.append([off, n])
            free.sort()
            merged = []
            for f in free:
                if merged and merged[-1][0] + merged[-1][1] == f[0]:
                    merged[-1][1] += f[1]
                else:
                    merged.append(f)
            free = merged
            out.append((2, 0, used))
    return out


def run_case(exe, L, om, H, blocks, betas, reach_prev, arena=(0, [])):
    N = L * L
    inp = struct.pack("<5I", L, len(blocks), len(betas), len(CUTS), reach_prev)
    inp += np.asarray(om, np.float64).tobytes() + np.asarray(H, np.uint64).tobytes()
    inp += np.asarray(blocks, np.uint64).tobytes() + np.asarray(betas, np.float64).tobytes()
    inp += np.asarray(CUTS, np.uint64).tobytes()
    size, ops = arena
    inp += struct.pack("<2Q", len(ops), size) + np.asarray(ops, np.uint64).reshape(-1).tobytes()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], input=inp, capture_output=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr.decode(errors="replace")[-2000:]
    rd = Reader(r.stdout)
    out = {"t5": rd.take(np.uint64, (N + 1) * 5), "t4": rd.take(np.uint64, (N + 1) * 4)}
    out["ok5"] = rd.one(np.uint32)
    out["f5"] = rd.take(np.uint32, (N + 1) * 5)
    out["ok8"] = rd.one(np.uint32)
    out["f8"] = rd.take(np.uint32, (N + 1) * 8)
    for k in ("flatness", "chebyshev", "kl"):
        out[k] = rd.one(np.float64)
    out["reach"], out["width"] = rd.one(np.int32), rd.one(np.int32)
    for norm in (0, 1):
        out["lg_rc%d" % norm] = rd.one(np.int32)
        out["lg%d" % norm] = rd.take(np.float64, N + 1)
    out["jk_rc"] = rd.one(np.int32)
    out["jk"], out["jk_err"] = rd.take(np.float64, N + 1), rd.take(np.float64, N + 1)
    out["can_rc"] = rd.one(np.int32)
    nb = len(betas)
    out["e"], out["e_err"] = rd.take(np.float64, nb), rd.take(np.float64, nb)
    out["c"], out["c_err"] = rd.take(np.float64, nb), rd.take(np.float64, nb)
    out["arena"] = [tuple(int(x) for x in rd.take(np.uint64, 2)) + (int(rd.one(np.uint64)),) for _ in ops]
    segs = []
    for _ in CUTS:
        n = rd.one(np.uint32)
        segs.append([(rd.take(np.uint64, 3), rd.take(np.uint32, 3)) for _ in range(n)])
    out["segs"] = segs
    assert rd.at == len(r.stdout)
    return out


def close(a, b, rel=1e-12):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    same_inf = (np.isinf(a) & np.isinf(b) & (np.sign(a) == np.sign(b))) | (np.isnan(a) & np.isnan(b))
    fin = np.isfinite(a) & np.isfinite(b)
    assert np.all(same_inf | fin), (a, b)
    assert np.all(np.abs(a[fin] - b[fin]) <= rel * np.maximum(1.0, np.abs(b[fin])))


def make_case(L, seed, kind):
    N = L * L
    rng = np.random.default_rng(seed)
    om = smooth_log_weights(L, seed) if kind != "random" else random_log_weights(L, seed, scale=30.0)
    blocks = rng.integers(0, 50, size=(5, N + 1)).astype(np.uint64)
    blocks[:, 1] = 0
    blocks[:, N - 1] = 0
    if kind == "holes":
        blocks[:, rng.integers(0, N + 1, size=N // 3)] = 0
        blocks[2, N // 2] = 7       # a bin present in one block only
        blocks[:, N // 2 + 1] = 0
    H = blocks.sum(axis=0)
    if kind == "empty-ground":
        H = H.copy()
        H[0] = 0
    return om, H, blocks


@pytest.mark.parametrize("L,seed,kind", [(4, 1, "smooth"), (6, 2, "random"), (34, 3, "holes"),
                                          (16, 4, "empty-ground"), (128, 5, "smooth")])
def test_host_math_under_sanitizers_matches_oracle(driver, L, seed, kind):
    N = L * L
    om, H, blocks = make_case(L, seed, kind)
    betas = [0.2, 0.4406868, 0.7]
    reach_prev = oracle.reachable_width(H) if kind != "random" else 3
    arena_size = 1 << 18 if seed % 2 else (1 << 18) + 4096 + 17  # not a multiple of 256 too
    ops = arena_ops(seed)
    out = run_case(driver, L, om, H, blocks, betas, reach_prev, (arena_size, ops))

    # the serving form's arena: exactly first fit with coalescing, and the
    # live ranges never overlap or leave the arena
    assert out["arena"] == model_arena(arena_size, ops)
    live = {}
    k = 0
    for (kind, a), (st, off, _) in zip(ops, out["arena"]):
        if kind == 0:
            if st == 1:
                n = -(-a // 256) * 256
                assert off % 256 == 0 and off + n <= arena_size
                assert all(off + n <= o or o + m <= off for o, m in live.values())
                live[k] = (off, n)
            k += 1
        else:
            live.pop(a, None)
    assert any(st == 0 for st, _, _ in out["arena"]) and any(st == 2 for st, _, _ in out["arena"])

    t5 = oracle.thresholds(N, om)
    np.testing.assert_array_equal(out["t5"], t5.reshape(-1))
    # kernel encodings: the four energy-changing moves by m = 0, 1, 3, 4, and
    # S = T - 1 for every move a configuration can propose (0 elsewhere)
    np.testing.assert_array_equal(out["t4"].reshape(N + 1, 4), t5[:, [4, 3, 1, 0]])
    proposable = np.zeros((N + 1, 5), bool)
    for k in range(N + 1):
        for m in range(5):
            kp = k + 2 - m
            proposable[k, m] = 0 <= kp <= N and k not in (1, N - 1) and kp not in (1, N - 1)
    t_by_m = t5[:, ::-1]
    ok = bool(np.all(t_by_m[proposable] > 0))
    assert bool(out["ok5"]) == ok and bool(out["ok8"]) == ok
    if ok:
        # slot 4 - m (= 2 + d for the bin change d = 2 - m of the move)
        want = np.where(proposable, t_by_m - 1, 0).astype(np.uint32)[:, ::-1]
        np.testing.assert_array_equal(out["f5"].reshape(N + 1, 5), want)
        f8 = out["f8"].reshape(N + 1, 8)
        np.testing.assert_array_equal(f8[:, :5], want)
        assert not f8[:, 5:].any()

    assert out["flatness"] == oracle.flatness(H)
    assert out["chebyshev"] == oracle.chebyshev(H)
    close(out["kl"], oracle.kl_divergence(H, reach_prev))
    assert out["reach"] == oracle.reachable_width(H) and out["width"] == oracle.width(H)
    for norm in (0, 1):
        ref = oracle.log_dos(H, om, norm)
        assert (out["lg_rc%d" % norm] == 0) == (ref is not None)
        if ref is not None:
            close(out["lg%d" % norm], ref)

    est, err = oan.jackknife_log_dos(list(blocks), om, norm=1)
    assert out["jk_rc"] == 0
    close(out["jk"], est, 1e-10)
    close(out["jk_err"], err, 1e-7)
    e, ee, c, ce = oan.canonical_jackknife(list(blocks), om, betas)
    assert out["can_rc"] == 0
    close(out["e"], e, 1e-10)
    close(out["c"], c, 1e-9)
    close(out["e_err"], ee, 1e-6)
    close(out["c_err"], ce, 1e-6)

    for (pos0, therm, rec), segs in zip(CUTS, out["segs"]):
        got = []
        for (sweep0, n, th), (sb, se, rb) in segs:
            if n:
                assert sb == se == rb == 0
                for t in range(int(n)):
                    got += [((sweep0 + t) * N + x, t >= th) for x in range(N)]
            else:
                assert sb < se <= N and sb <= rb <= se
                got += [(sweep0 * N + x, x >= rb) for x in range(sb, se)]
        want = [(p, p >= pos0 + therm) for p in range(pos0, pos0 + therm + rec)]
        assert got == want, (pos0, therm, rec)
