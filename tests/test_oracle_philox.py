"""Pins for the oracle's Philox4x32-10 (the generator of Sec. 2.3).

The oracle writes Philox4x32-10 out from its published definition
(Salmon et al. 2011).  It is checked against an implementation it shares no
code with -- the open-source rocRAND header shipped with ROCm, compiled here
for the host only by a throw-away program in a temporary directory -- and by
simple statistical properties of the outputs.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROCRAND_HEADER = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

XCHECK_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct probe : rocrand_device::philox4x32_10_engine {
    static uint4 block(uint4 c, uint2 k) { probe p; return p.ten_rounds(c, k); }
};
int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = probe::block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
"""


def _cases():
    rng = np.random.default_rng(2017)
    cases = [
        [0, 0, 0, 0, 0, 0],
        [0xFFFFFFFF] * 6,
        [1, 0, 0, 0, 0, 0],
        [0, 0, 0, 1, 7, 3],
        [5, 200, 0, 0, 1, 16383],
    ]
    cases += rng.integers(0, 2 ** 32, size=(60, 6), dtype=np.uint64).tolist()
    return [[int(v) for v in c] for c in cases]


def test_philox_matches_rocrand_header(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(ROCRAND_HEADER) or not os.path.exists(hipcc):
        pytest.skip("rocRAND header or hipcc not available")
    src = tmp_path / "xcheck.cpp"
    src.write_text(XCHECK_SRC)
    exe = tmp_path / "xcheck"
    subprocess.run([hipcc, "-O1", str(src), "-o", str(exe)], check=True,
                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    cases = _cases()
    stdin = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([str(exe)], input=stdin, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        ref = [int(v) for v in line.split()]
        got = oracle.philox4x32_10(c[:4], c[4:]).tolist()
        assert got == ref, (c, got, ref)


def test_draw_is_word_of_block():
    # site i uses word i & 3 of the block with counter word 0 = i >> 2
    for site in range(8):
        blk = oracle.philox4x32_10([site >> 2, 5, 0, 0], [9, 3])
        assert oracle.draw(9, 3, 5, site, 0) == int(blk[site & 3])
    big = (7 << 32) | 11
    blk = oracle.philox4x32_10([2, 11, 7, 0], [1, 2])
    assert oracle.draw(1, 2, big, 9, 0) == int(blk[1])


def _draws(n_walkers=256, n_sites=256, seed=1, sweep=0, domain=0):
    return np.array([oracle.draw(seed, w, sweep, i, domain)
                     for w in range(n_walkers) for i in range(n_sites)], dtype=np.uint64)


def test_bit_balance_and_top_byte():
    u = _draws()
    n = u.size
    for b in range(32):
        frac = float(((u >> np.uint64(b)) & np.uint64(1)).mean())
        assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(n), (b, frac)
    top = (u >> np.uint64(24)).astype(np.int64)
    counts = np.bincount(top, minlength=256)
    expected = n / 256.0
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    assert chi2 < 255 + 6 * np.sqrt(2 * 255), chi2


def test_streams_are_distinct():
    a = _draws(8, 64, seed=1)
    b = _draws(8, 64, seed=2)
    c = _draws(8, 64, seed=1, sweep=1)
    d = _draws(8, 64, seed=1, domain=1)
    for x, y in [(a, b), (a, c), (a, d)]:
        assert np.count_nonzero(x == y) < 3
    # walkers differ from each other
    w = a.reshape(8, 64)
    for i in range(8):
        for j in range(i + 1, 8):
            assert np.count_nonzero(w[i] == w[j]) < 3
