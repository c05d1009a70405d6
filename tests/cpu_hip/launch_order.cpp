// Checks the launch order of batched rounds (muca_batch.cpp, muca_order.hip)
// on the CPU stand-in for HIP: the two-wave launches are issued before the
// others, each kind by its longest chain, and in rounds that are crowded or
// run pair workgroups each launch after the first waits 30 us more than the one
// before (up to eight steps); rounds that fit without pairs start every launch
// at once.  Test infrastructure only.  Prints "ok" at the end.
#include <cstdio>
#include <vector>

#include "muca.h"

struct CpuHipLaunch {
    const void* stream;
    int form;
    uint32_t value;
};
std::vector<CpuHipLaunch> cpu_hip_take_launch_log();

namespace {

struct Member {
    uint32_t L, walkers;
};

bool two_wave(int form) { return form == 2 || form == 4 || form == 5; }

int fail(const char* round, const char* what)
{
    std::printf("FAIL %s: %s\n", round, what);
    return 1;
}

// One round of every member iterating `sweeps` sweeps; checks the logged launches.
int check(const char* name, const std::vector<Member>& ms, uint32_t flags, bool stagger, int first_form)
{
    std::vector<muca_instance*> hs;
    for (size_t i = 0; i < ms.size(); ++i) {
        muca_params p{ms[i].L, ms[i].walkers, (uint32_t)(100 + i), 0};
        muca_instance* h = nullptr;
        if (muca_create(&p, nullptr, nullptr, 0, &h) != MUCA_OK)
            return fail(name, "muca_create");
        hs.push_back(h);
    }
    muca_batch* b = nullptr;
    if (muca_batch_create(hs.data(), (uint32_t)hs.size(), nullptr, flags, &b) != MUCA_OK)
        return fail(name, "muca_batch_create");
    cpu_hip_take_launch_log();
    std::vector<uint32_t> mode(ms.size(), MUCA_BATCH_ITERATE), therm(ms.size(), 0), sweeps(ms.size(), 2);
    std::vector<muca_info> infos(ms.size());
    if (muca_batch_run(b, mode.data(), therm.data(), sweeps.data(), infos.data()) != MUCA_OK)
        return fail(name, muca_batch_last_error(b));
    const std::vector<CpuHipLaunch> log = cpu_hip_take_launch_log();
    // pair each sweep launch with the wait issued on its stream just before it
    std::vector<CpuHipLaunch> launches;
    std::vector<uint32_t> waits;
    for (size_t k = 0; k < log.size(); ++k) {
        if (log[k].form < 0)
            continue;
        uint32_t wait = 0;
        for (size_t j = k; j-- > 0;) {
            if (log[j].stream != log[k].stream)
                continue;
            if (log[j].form < 0)
                wait = log[j].value;
            break;
        }
        launches.push_back(log[k]);
        waits.push_back(wait);
    }
    if (launches.size() < 2)
        return fail(name, "fewer than two launches");
    if (launches[0].form != first_form)
        return fail(name, "unexpected first launch");
    for (size_t k = 1; k < launches.size(); ++k) {
        const CpuHipLaunch& p = launches[k - 1];
        const CpuHipLaunch& q = launches[k];
        if (!two_wave(p.form) && two_wave(q.form))
            return fail(name, "a two-wave launch after a one-wave one");
        // every member runs the same sweeps, so the chain order is the L order
        if (two_wave(p.form) == two_wave(q.form) && q.value > p.value)
            return fail(name, "a longer chain launched after a shorter one of its kind");
    }
    for (size_t k = 0; k < launches.size(); ++k) {
        const uint32_t want = stagger ? 30u * (uint32_t)(k < 8 ? k : 8) : 0u;
        if (waits[k] != want) {
            std::printf("FAIL %s: launch %zu (form %d, L %u) waits %u us, expected %u\n", name, k, launches[k].form,
                        launches[k].value, waits[k], want);
            return 1;
        }
    }
    muca_batch_destroy(b);
    for (muca_instance* h : hs)
        muca_destroy(h);
    std::printf("%s: %zu launches, first form %d, last wait %u us\n", name, launches.size(), launches[0].form,
                waits.back());
    return 0;
}

}  // namespace

int main()
{
    // crowded (540 blocks on 256 CUs): the mixed-longest shape gives the two-wave
    // form to the L = 96 member alone; the one-wave groups follow, L = 64 first
    const std::vector<Member> crowded = {{64, 16448}, {48, 16448}, {8, 300}, {16, 1000}, {96, 65}, {32, 130}};
    // pairs: single two-wave workgroups do not all fit, pairs do
    const std::vector<Member> paired = {{64, 16448}, {8, 300}, {16, 1000}};
    // everything fits without pairs
    const std::vector<Member> fits = {{8, 300}, {16, 1000}, {32, 130}, {24, 700}};
    for (uint32_t flags : {0u, (uint32_t)MUCA_BATCH_GRAPH}) {
        if (check(flags ? "crowded, graph" : "crowded", crowded, flags, true, 4) ||
            check(flags ? "paired, graph" : "paired", paired, flags, true, 5) ||
            check(flags ? "fits, graph" : "fits", fits, flags, false, 2))
            return 1;
    }
    std::printf("ok\n");
    return 0;
}
