// muca_host_math.cpp -- the host arithmetic of libmuca that needs no device:
// acceptance thresholds from the log weights and their kernel encodings, the
// histogram statistics, ln g, and the cut of a call into sweep segments.
// Kept free of HIP so that it can also be built alone (with the sanitizers,
// in the CPU tests).
#include "muca_host_math.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace muca_host {

// Acceptance thresholds (Sec. 2.3 acceptance min(1, exp[omega(E') - omega(E)])
// as an integer bound on a uint32 draw): T[k*5+d], k' = k + d - 2.
void compute_thresholds(uint32_t N, const double* om, uint64_t* t5)
{
    const uint64_t always = (uint64_t)1 << 32;
    for (uint32_t k = 0; k <= N; ++k) {
        for (int d = 0; d < 5; ++d) {
            const long kp = (long)k + d - 2;
            uint64_t t = 0;
            if (kp >= 0 && kp <= (long)N) {
                const double diff = om[kp] - om[k];
                if (om[kp] >= om[k])
                    t = always;
                else
                    t = (uint64_t)std::floor(std::ldexp(std::exp(diff), 32));
            }
            t5[(size_t)k * 5 + d] = t;
        }
    }
}

// Device table: the four energy-changing moves per bin, ordered by the number
// m of anti-aligned neighbours (m = 0, 1, 3, 4 <-> d = 4, 3, 1, 0).
void device_table(uint32_t N, const uint64_t* t5, uint64_t* t4)
{
    static const int kDofSlot[4] = {4, 3, 1, 0};
    for (uint32_t k = 0; k <= N; ++k)
        for (int s = 0; s < 4; ++s)
            t4[(size_t)k * 4 + s] = t5[(size_t)k * 5 + kDofSlot[s]];
}

// Fast-kernel table: S = T - 1 as uint32 for every move out of bin k, indexed
// by the count m = 0..4 of anti-aligned neighbours (d = 4 - m).  A move can be
// proposed only between energies some configuration has: never to a target
// outside 0..N, and never from or to the forbidden bins 1 and N-1 (no
// configuration has E = -(2N-4) or 2N-4, Sec. 3).  Those entries are never
// read and get 0.  Returns false when a move that can be proposed has T = 0:
// r <= T - 1 cannot express "never", so the generic kernel must run.
bool fast_table(uint32_t N, const uint64_t* t5, uint32_t* f, uint32_t stride)
{
    for (uint32_t k = 0; k <= N; ++k) {
        for (uint32_t m = 5; m < stride; ++m)
            f[(size_t)k * stride + m] = 0u;
        for (int m = 0; m < 5; ++m) {
            const long kp = (long)k + 2 - m;
            const uint64_t t = t5[(size_t)k * 5 + (4 - m)];
            if (kp < 0 || kp > (long)N || k == 1 || k == N - 1 || kp == 1 || kp == (long)N - 1) {
                f[(size_t)k * stride + (4 - m)] = 0u;
                continue;
            }
            if (t == 0)
                return false;
            f[(size_t)k * stride + (4 - m)] = (uint32_t)(t - 1);
        }
    }
    return true;
}

static bool reachable(uint32_t N, uint32_t k) { return k != 1 && k != N - 1; }

double flatness_of(uint32_t N, const uint64_t* H)
{
    uint64_t sum = 0, mn = std::numeric_limits<uint64_t>::max();
    for (uint32_t k = 0; k <= N; ++k) {
        if (!reachable(N, k))
            continue;
        sum += H[k];
        if (H[k] < mn)
            mn = H[k];
    }
    if (sum == 0)
        return 0.0;
    const double mean = (double)sum / (double)(N - 1);
    return (double)mn / mean;
}

double chebyshev_of(uint32_t N, const uint64_t* H)
{
    uint64_t sum = 0;
    for (uint32_t k = 0; k <= N; ++k)
        if (reachable(N, k))
            sum += H[k];
    if (sum == 0)
        return 0.0;
    const double m = (double)sum / (double)(N - 1);
    double worst = 0.0;
    for (uint32_t k = 0; k <= N; ++k) {
        if (!reachable(N, k))
            continue;
        const double dev = std::fabs((double)H[k] / m - 1.0);
        if (dev > worst)
            worst = dev;
    }
    return worst;
}

double kl_of(uint32_t N, const uint64_t* H, int reach_prev)
{
    uint64_t sum = 0;
    for (uint32_t k = 0; k <= N; ++k)
        sum += H[k];
    if (sum == 0)
        return 0.0;
    const double w = (double)(reach_prev > 10 ? reach_prev : 10);
    double dk = 0.0;
    for (uint32_t k = 0; k <= N; ++k) {
        if (H[k] == 0)
            continue;
        const double p = (double)H[k] / (double)sum;
        dk += p * std::log(p * w);
    }
    return dk;
}

int reach_of(uint32_t N, const uint64_t* H)
{
    int lo = -1, hi = -1;
    for (uint32_t k = 0; k <= N; ++k)
        if (H[k] > 0) {
            if (lo < 0)
                lo = (int)k;
            hi = (int)k;
        }
    int n = 0;
    for (int k = lo; lo >= 0 && k <= hi; ++k)
        n += (k != 1 && k != (int)N - 1) ? 1 : 0;
    return n;
}

int width_of(uint32_t N, const uint64_t* H)
{
    int lo = -1, hi = -1;
    for (uint32_t k = 0; k <= N; ++k) {
        if (H[k] > 0) {
            if (lo < 0)
                lo = (int)k;
            hi = (int)k;
        }
    }
    return lo < 0 ? 0 : hi - lo + 1;
}

int log_dos_of(uint32_t N, const uint64_t* H, const double* omega, int normalization, double* out)
{
    double mx = -INFINITY;
    for (uint32_t k = 0; k <= N; ++k) {
        if (k != 1 && k != N - 1 && H[k] > 0) {
            out[k] = std::log((double)H[k]) - omega[k];
            if (out[k] > mx)
                mx = out[k];
        } else {
            out[k] = -INFINITY;
        }
    }
    double c;
    if (normalization == 0) {
        if (H[0] == 0)
            return 1;
        c = std::log(2.0) - out[0];
    } else {
        if (mx == -INFINITY)
            return 2;
        double s = 0.0;
        for (uint32_t k = 0; k <= N; ++k)
            if (out[k] != -INFINITY)
                s += std::exp(out[k] - mx);
        c = (double)N * std::log(2.0) - (mx + std::log(s));
    }
    for (uint32_t k = 0; k <= N; ++k)
        if (out[k] != -INFINITY)
            out[k] += c;
    return 0;
}

// Cuts the attempts [pos0, pos0 + therm + recorded) -- recording from
// pos0 + therm on -- into whole-sweep runs for the sweep kernels and partial
// sweeps for the range kernel.  A sweep that holds the start of recording is
// run as a partial sweep unless recording starts at its first site.
std::vector<Segment> segments_of(uint64_t N, uint64_t pos0, uint64_t therm, uint64_t recorded)
{
    std::vector<Segment> out;
    const uint64_t rec = pos0 + therm, end = rec + recorded;
    uint64_t p = pos0;
    while (p < end) {
        const uint64_t sweep = p / N, base = sweep * N;
        const uint64_t sweep_end = base + N;
        const bool partial = p != base || end < sweep_end || (rec > p && rec < sweep_end);
        if (partial) {
            const uint64_t e = std::min(end, sweep_end);
            const uint64_t rb = std::min(std::max(rec, p), e);
            out.push_back(Segment{sweep, 0, 0, (uint32_t)(p - base), (uint32_t)(e - base),
                                  (uint32_t)(rb - base)});
            p = e;
            continue;
        }
        // whole sweeps up to the end, or up to the sweep holding the start of
        // recording when that start is not on a sweep boundary
        uint64_t n = (end - p) / N;
        if (rec > p && (rec - p) % N != 0)
            n = std::min(n, (rec - p) / N);
        const uint64_t th = rec > p ? std::min(n, (rec - p) / N) : 0;
        out.push_back(Segment{sweep, n, th, 0, 0, 0});
        p += n * N;
    }
    return out;
}

double solve_work_estimate(uint32_t L, uint32_t walkers, uint32_t iter_therm, uint32_t iter_sweeps,
                           uint32_t max_iterations, uint32_t prod_therm, uint32_t prod_sweeps)
{
    const double n = (double)L * L;
    double iterations = std::max(1.0, n / 20.0);
    if (max_iterations)
        iterations = std::min(iterations, (double)max_iterations);
    const double sweeps = iterations * ((double)iter_therm + iter_sweeps) + prod_therm + prod_sweeps;
    return (double)walkers * n * sweeps;
}

RoundFit round_fit(const RoundMember* m, size_t n, uint32_t cus, uint32_t lds_per_cu)
{
    RoundFit fit;
    fit.share.assign(n, 0.0);
    fit.pairable.assign(n, 0);
    std::vector<double>& share = fit.share;
    uint64_t blocks = 0;
    double single = 0.0, paired = 0.0;
    std::vector<double> share_pair(n, 0.0);
    for (size_t i = 0; i < n; ++i) {
        if (!m[i].active)
            continue;
        fit.walkers += m[i].walkers;
        blocks += m[i].blocks;
        const double nb = (double)m[i].blocks;
        const bool two_capable = (m[i].table == kFormFast && m[i].split_ok) ||
                                 (m[i].table == kFormWide && m[i].wide_split_ok);
        if (two_capable && m[i].two_wave_bytes > 0 && m[i].two_wave_bytes <= lds_per_cu)
            share[i] = nb * std::max(0.5, 1.0 / (double)(lds_per_cu / m[i].two_wave_bytes));
        share_pair[i] = share[i];
        if (m[i].table == kFormFast && m[i].pair_ok && !m[i].forced_fast && share[i] > 0.0 &&
            lds_per_cu / m[i].two_wave_bytes == 1u) {
            fit.pairable[i] = 1;
            share_pair[i] = 0.5 * nb;
        }
        single += share[i];
        paired += share_pair[i];
    }
    const bool fits_blocks = blocks <= 2u * (uint64_t)cus;
    fit.two_wave_single = fits_blocks && single <= (double)cus;
    fit.two_wave = fit.two_wave_single || (fits_blocks && paired <= (double)cus);
    fit.use_pairs = !fit.two_wave_single;
    if (fit.use_pairs)
        for (size_t i = 0; i < n; ++i)
            share[i] = share_pair[i];
    return fit;
}

void plan_forms(const RoundMember* m, size_t n, uint32_t cus, const RoundFit& fit, int shape, uint32_t* form,
                uint32_t* waves)
{
    const std::vector<double>& share = fit.share;
    std::vector<char> two(n, 0);
    if (shape == kShapeTwoWave) {
        std::fill(two.begin(), two.end(), 1);
    } else if (shape == kShapeMixed || shape == kShapeMixedLongest) {
        std::vector<size_t> order;
        for (size_t i = 0; i < n; ++i)
            if (m[i].active && share[i] > 0.0)
                order.push_back(i);
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
            return m[x].chain != m[y].chain ? m[x].chain > m[y].chain : m[x].walkers < m[y].walkers;
        });
        double used = 0.0;
        uint64_t blocks = 0;
        for (size_t i : order) {
            // mixed-longest: the two-wave form for the longest chains alone, so
            // that the shorter ones start at once on the CUs left over
            if (shape == kShapeMixedLongest && m[i].chain < m[order.front()].chain)
                break;
            if (used + share[i] > (double)cus || blocks + m[i].blocks > 2u * (uint64_t)cus)
                break;
            used += share[i];
            blocks += m[i].blocks;
            two[i] = 1;
        }
    }
    for (size_t i = 0; i < n; ++i) {
        form[i] = kFormGeneric;
        waves[i] = 1u;
        if (!m[i].active)
            continue;
        form[i] = m[i].table;
        if (m[i].table == kFormWide && two[i] && !m[i].forced_fast && m[i].wide_split_ok)
            form[i] = kFormWideSplit;  // the same tables, Philox on a second wave
        if (m[i].table == kFormFast) {
            const bool want_fast = m[i].forced_fast || !two[i];
            if (two[i] && fit.use_pairs && fit.pairable[i]) {
                form[i] = kFormPair;
                waves[i] = 2u;  // two chains count into one table
            } else if (m[i].split_ok && !(want_fast && m[i].fast_ok)) {
                form[i] = kFormSplit;
            } else {
                form[i] = kFormFast;
                waves[i] = shape == kShapeOneWaveFour ? 4u : m[i].fast_waves;
            }
        }
    }
}

size_t admission_pick(const QueuedJob* q, size_t n, bool smallest_first, double now, double max_wait_s)
{
    if (n == 0 || !smallest_first)
        return 0;
    for (size_t i = 0; i < n; ++i)  // arrival order: the first overdue one is the oldest
        if (now - q[i].t_submit > max_wait_s)
            return i;
    size_t best = 0;
    for (size_t i = 1; i < n; ++i)
        if (q[i].work < q[best].work)
            best = i;
    return best;
}

}  // namespace muca_host
