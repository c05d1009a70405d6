// Drives libmuca's server (include/muca.h, muca_server_*) through a stream of
// requests on the CPU stand-in for HIP, the way the serving benchmark does:
// submissions at their arrival times, progress() between them, every
// finished request taken.  Built with the library's host sources and
// cpu_hip.cpp under the sanitizers; test infrastructure only.
//
//   served_stream REQUESTS MEM_CAP_BYTES MAX_WALKERS BATCH_FLAGS POLICY TIME_SCALE SOLO_EVERY
//
// REQUESTS holds one request per line: arrival_s L walkers seed.  Arrival
// times are divided by TIME_SCALE.  Each result is checked against what the
// stand-in kernels make of it (status, weight iterations, attempts, finite
// ln g), and every SOLO_EVERY-th request is solved again alone
// (muca_create / muca_iterate / muca_production / muca_log_dos) and its ln g
// compared bit for bit with the served one.  Prints "ok <requests>" at the end.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <thread>
#include <vector>

#include "muca.h"

uint64_t cpu_hip_free_waits();

namespace {

struct Req {
    double t;
    uint32_t L, W, seed;
};

constexpr uint32_t kIterSweeps = 200, kProdTherm = 2000, kProdSweeps = 2000, kMaxIter = 2000;
constexpr double kMinFlat = 0.5;

// Weight iterations the stand-in kernels take to a flat histogram: iteration
// i (from 1) fills the first 16 * 2^(i - 1) bins.
uint32_t expected_iterations(uint32_t L)
{
    const uint64_t N1 = (uint64_t)L * L + 1;
    uint32_t i = 1;
    while ((16ull << (i - 1)) < N1)
        ++i;
    return i;
}

int fail(const char* what, uint64_t i)
{
    std::printf("FAIL request %llu: %s\n", (unsigned long long)i, what);
    std::fflush(stdout);
    return 1;
}

bool solo(const Req& r, std::vector<double>& ln_g)
{
    muca_params p{r.L, r.W, r.seed, 0};
    muca_instance* h = nullptr;
    if (muca_create(&p, nullptr, nullptr, 0, &h) != MUCA_OK)
        return false;
    muca_info info{};
    bool ok = true;
    for (uint32_t it = 0; it < kMaxIter; ++it) {
        if (muca_iterate(h, 0, kIterSweeps, &info) != MUCA_OK) {
            ok = false;
            break;
        }
        if (info.flatness >= kMinFlat)
            break;
    }
    ok = ok && muca_production(h, kProdTherm, kProdSweeps, &info) == MUCA_OK;
    ln_g.assign((size_t)r.L * r.L + 1, 0.0);
    ok = ok && muca_log_dos(h, 0, ln_g.data(), ln_g.size()) == MUCA_OK;
    muca_destroy(h);
    return ok;
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc != 8) {
        std::fprintf(stderr, "usage: %s REQUESTS MEM_CAP MAX_WALKERS BATCH_FLAGS POLICY TIME_SCALE SOLO_EVERY\n",
                     argv[0]);
        return 2;
    }
    std::vector<Req> reqs;
    {
        FILE* f = std::fopen(argv[1], "r");
        if (!f)
            return 2;
        Req r;
        while (std::fscanf(f, "%lf %u %u %u", &r.t, &r.L, &r.W, &r.seed) == 4)
            reqs.push_back(r);
        std::fclose(f);
    }
    muca_server_config cfg{};
    cfg.mem_cap_bytes = std::strtoull(argv[2], nullptr, 10);
    cfg.max_active_walkers = std::strtoull(argv[3], nullptr, 10);
    cfg.batch_flags = (uint32_t)std::atoi(argv[4]);
    cfg.policy = (uint32_t)std::atoi(argv[5]);
    cfg.max_wait_s = 0.0;
    const double scale = std::atof(argv[6]);
    const uint32_t solo_every = (uint32_t)std::atoi(argv[7]);

    muca_server* s = nullptr;
    if (muca_server_create(&cfg, &s) != MUCA_OK) {
        std::printf("FAIL server create: %s\n", muca_server_last_error(nullptr));
        return 1;
    }
    std::map<uint64_t, size_t> tickets;  // ticket -> request
    std::map<size_t, std::vector<double>> served_lng;
    size_t next = 0, done = 0;
    const auto t0 = std::chrono::steady_clock::now();
    auto last_note = t0;
    while (done < reqs.size()) {
        const double now = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        while (next < reqs.size() && reqs[next].t / scale <= now) {
            const Req& r = reqs[next];
            muca_request q{};
            q.min_flatness = kMinFlat;
            q.L = r.L;
            q.walkers = r.W;
            q.seed = r.seed;
            q.iter_sweeps = kIterSweeps;
            q.max_iterations = kMaxIter;
            q.prod_therm = kProdTherm;
            q.prod_sweeps = kProdSweeps;
            uint64_t t = 0;
            if (muca_server_submit(s, &q, &t) != MUCA_OK)
                return fail(muca_server_last_error(s), next);
            tickets[t] = next++;
        }
        uint32_t ev = 0;
        if (muca_server_progress(s, &ev) != MUCA_OK)
            return fail(muca_server_last_error(s), done);
        if (ev == 0)
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        for (auto it = tickets.begin(); it != tickets.end();) {
            const size_t i = it->second;
            const Req& r = reqs[i];
            std::vector<double> lng((size_t)r.L * r.L + 1);
            muca_result res{};
            const int rc = muca_server_take(s, it->first, &res, lng.data(), lng.size());
            if (rc == MUCA_PENDING) {
                ++it;
                continue;
            }
            if (rc != MUCA_OK)
                return fail(muca_server_last_error(s), i);
            if (res.status != MUCA_OK)
                return fail("status is not MUCA_OK", i);
            if (res.iterations != expected_iterations(r.L))
                return fail("weight iterations differ from the stand-in's", i);
            const uint64_t N = (uint64_t)r.L * r.L;
            if (res.attempts != (uint64_t)r.W * N * (res.iterations * kIterSweeps + kProdTherm + kProdSweeps))
                return fail("attempts differ", i);
            for (uint64_t k = 0; k <= N; ++k)
                if (k != 1 && k != N - 1 && !std::isfinite(lng[k]))
                    return fail("ln g not finite", i);
            if (solo_every && i % solo_every == 0)
                served_lng[i] = lng;
            ++done;
            it = tickets.erase(it);
        }
        const auto tn = std::chrono::steady_clock::now();
        if (std::chrono::duration<double>(tn - last_note).count() > 10.0) {
            muca_server_counters c{};
            muca_server_stats(s, &c);
            std::printf("served %zu/%zu, active %u, queued %u, %.0f s\n", done, reqs.size(), c.active, c.queued,
                        c.clock_s);
            std::fflush(stdout);
            last_note = tn;
        }
    }
    muca_server_destroy(s);
    for (auto& kv : served_lng) {
        std::vector<double> lng;
        if (!solo(reqs[kv.first], lng))
            return fail("solo solve failed", kv.first);
        if (std::memcmp(lng.data(), kv.second.data(), lng.size() * sizeof(double)) != 0)
            return fail("served ln g differs from the solo solve", kv.first);
    }
    std::printf("ok %zu solo %zu free_waits %llu\n", reqs.size(), served_lng.size(),
                (unsigned long long)cpu_hip_free_waits());
    return 0;
}
