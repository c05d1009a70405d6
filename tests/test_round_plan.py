"""The batch runtime's launch planning (muca_host::round_fit and plan_forms in
csrc/muca_host_math.cpp) built alone with AddressSanitizer and
UndefinedBehaviourSanitizer and run over seeded random rounds: members of
every table kind, capability, size and sweep count (every L with a record
table has the one-wave kernel, as in the library), on devices of 1 to 256
CUs, in every launch shape.  No device is involved.

Checked for every round against the planner's stated rules:

* every member gets a form its table and its L allow, and the waves per
  workgroup that form runs with (pairs 2, the one-wave form its default or 4);
* a skipped member gets nothing;
* when the round fits and the shape is two-wave, every member with a two-wave
  form runs it (in pairs only where single workgroups do not fit);
* in the mixed shapes the two-wave members fit (shares <= CUs, blocks <= 2 per
  CU), and none of them ranks after a member left one-wave in the order the
  rule gives (longest chain first, then fewest walkers); in the mixed-longest
  shape every two-wave member's chain is the round's longest.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
CSRC = os.path.join(ROOT, "paper_1707_00919_amd", "csrc")

FUZZ = r"""
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "muca_host_math.h"

using namespace muca_host;

static uint64_t state = 0x9e3779b97f4a7c15ull;
static uint64_t next()
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}
static uint32_t below(uint32_t n) { return (uint32_t)(next() % n); }

#define CHECK(c)                                                                      \
    do {                                                                              \
        if (!(c)) {                                                                   \
            std::printf("FAIL round %d member %zu: %s\n", round, i, #c);             \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

int main(int argc, char** argv)
{
    const int rounds = argc > 1 ? std::atoi(argv[1]) : 20000;
    const uint32_t lds = 160u * 1024u;
    const uint32_t cus_choices[] = {1, 4, 32, 256};
    const int shapes[] = {kShapeTwoWave, kShapeOneWave, kShapeOneWaveFour, kShapeMixed, kShapeMixedLongest};
    size_t i = 0;
    uint64_t seen[6] = {0, 0, 0, 0, 0, 0}, fits = 0, single = 0, seen_longest[2] = {0, 0};
    for (int round = 0; round < rounds; ++round) {
        const size_t n = below(60);
        const uint32_t cus = cus_choices[below(4)];
        std::vector<RoundMember> m(n);
        for (i = 0; i < n; ++i) {
            RoundMember& r = m[i];
            r.active = below(8) != 0;
            r.L = 4 + 2 * below(63);
            r.blocks = 1 + below(below(4) == 0 ? 2000 : 40);
            r.walkers = 64 * r.blocks - below(64);
            r.chain = (uint64_t)r.L * r.L * (1 + below(300));
            const uint32_t t = below(3);
            r.table = t == 0 ? kFormGeneric : (t == 1 ? kFormFast : kFormWide);
            r.forced_fast = below(6) == 0;
            r.split_ok = below(5) != 0;
            r.fast_ok = true;  // every L with a record table has the one-wave kernel
            r.pair_ok = r.split_ok && below(3) == 0;
            r.wide_split_ok = below(4) != 0;
            r.two_wave_bytes = below(5) == 0 ? 0u : 1024u + below(lds);
            r.fast_waves = 1u << below(3);
        }
        const RoundFit fit = round_fit(m.data(), n, cus, lds);
        i = 0;
        CHECK(fit.share.size() == n && fit.pairable.size() == n);
        CHECK(!fit.two_wave_single || fit.two_wave);
        CHECK(fit.use_pairs == !fit.two_wave_single);
        fits += fit.two_wave;
        single += fit.two_wave_single;
        for (int shape : shapes) {
            std::vector<uint32_t> form(n, 77u), waves(n, 77u);
            plan_forms(m.data(), n, cus, fit, shape, form.data(), waves.data());
            const bool mixed = shape == kShapeMixed || shape == kShapeMixedLongest;
            uint64_t longest = 0;
            for (i = 0; i < n; ++i)
                if (m[i].active && fit.share[i] > 0.0)
                    longest = longest > m[i].chain ? longest : m[i].chain;
            double used = 0.0;
            uint64_t blocks = 0;
            for (i = 0; i < n; ++i) {
                const RoundMember& r = m[i];
                if (!r.active) {
                    CHECK(form[i] == kFormGeneric && waves[i] == 1u);
                    continue;
                }
                const uint32_t f = form[i];
                CHECK(f < 6u);
                ++seen[f];
                if (r.table == kFormGeneric)
                    CHECK(f == kFormGeneric && waves[i] == 1u);
                if (r.table == kFormWide) {
                    CHECK(f == kFormWide || f == kFormWideSplit);
                    CHECK(f != kFormWideSplit || (r.wide_split_ok && !r.forced_fast));
                    CHECK(waves[i] == 1u);
                }
                if (r.table == kFormFast) {
                    CHECK(f == kFormFast || f == kFormSplit || f == kFormPair);
                    CHECK(f != kFormSplit || r.split_ok);
                    CHECK(f != kFormFast || r.fast_ok || !r.split_ok);
                    CHECK(f != kFormPair || (fit.use_pairs && fit.pairable[i] && r.pair_ok && !r.forced_fast));
                    CHECK(f != kFormPair || waves[i] == 2u);
                    CHECK(f != kFormSplit || waves[i] == 1u);
                    CHECK(f != kFormFast || waves[i] == (shape == kShapeOneWaveFour ? 4u : r.fast_waves));
                    if (shape == kShapeOneWave || shape == kShapeOneWaveFour)
                        CHECK(f == kFormFast || !r.fast_ok);
                    if (r.forced_fast && r.fast_ok)
                        CHECK(f == kFormFast);
                }
                const bool two = f == kFormSplit || f == kFormWideSplit || f == kFormPair;
                if (shape == kShapeTwoWave && fit.two_wave && fit.share[i] > 0.0 && !r.forced_fast)
                    CHECK(two);
                if (mixed && two && fit.share[i] > 0.0) {
                    used += fit.share[i];
                    blocks += r.blocks;
                    if (shape == kShapeMixedLongest)
                        CHECK(r.chain == longest);
                    ++seen_longest[shape == kShapeMixedLongest];
                }
            }
            if (mixed) {
                i = 0;
                CHECK(used <= (double)cus + 1e-9);
                CHECK(blocks <= 2ull * cus);
                // no two-wave member ranks after a one-wave one
                for (i = 0; i < n; ++i) {
                    if (!m[i].active || fit.share[i] <= 0.0)
                        continue;
                    // a member held to the one-wave form by its flag may have been given room
                    const bool ti = form[i] == kFormSplit || form[i] == kFormWideSplit || form[i] == kFormPair ||
                                    m[i].forced_fast;
                    if (ti)
                        continue;
                    for (size_t j = 0; j < n; ++j) {
                        if (!m[j].active || fit.share[j] <= 0.0 || j == i)
                            continue;
                        const bool tj = form[j] == kFormSplit || form[j] == kFormWideSplit || form[j] == kFormPair;
                        const bool j_after_i = m[j].chain != m[i].chain ? m[j].chain < m[i].chain
                                               : m[j].walkers != m[i].walkers ? m[j].walkers > m[i].walkers
                                                                              : j > i;
                        if (tj && j_after_i) {
                            std::printf("FAIL round %d: member %zu two-wave but ranks after one-wave %zu\n", round,
                                        j, i);
                            return 1;
                        }
                    }
                }
            }
        }
    }
    std::printf("ok %d", rounds);
    for (uint64_t c : seen)
        std::printf(" %llu", (unsigned long long)c);
    std::printf(" %llu %llu %llu %llu\n", (unsigned long long)fits, (unsigned long long)single,
                (unsigned long long)seen_longest[0], (unsigned long long)seen_longest[1]);
    return 0;
}
"""


@pytest.fixture(scope="module")
def fuzz(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("round_plan")
    src = d / "fuzz.cpp"
    src.write_text(FUZZ)
    exe = d / "round_plan"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(CSRC, "muca_host_math.cpp"), str(src), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    return str(exe)


def test_round_plan_rules_hold_over_random_rounds(fuzz):
    r = subprocess.run([fuzz, "20000"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-2000:]
    words = r.stdout.split()
    assert words[:2] == ["ok", "20000"]
    seen = [int(w) for w in words[2:8]]
    fits, single = int(words[8]), int(words[9])
    two_wave_mixed, two_wave_longest = int(words[10]), int(words[11])
    # every form came up, and rounds that fit with single workgroups, only in
    # pairs, and not at all; both mixed shapes gave some members the two-wave
    # form, the mixed-longest shape to fewer
    assert all(c > 0 for c in seen), seen
    assert 0 < single < fits < 20000
    assert 0 < two_wave_longest < two_wave_mixed
