// muca_runtime.cpp -- host side of libmuca: the C ABI declared in
// include/muca.h.  Owns the instance state, computes the acceptance
// thresholds from the log weights, drives the device kernels on the
// instance's stream, and applies the weight recursion of Eq. 4 on the host
// (Sec. 2.2: the summed histogram defines the next weights, which are then
// handed to every walker).
#include "muca.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "muca_device.h"
#include "muca_internal.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool params_valid(const muca_params* p, std::string* why)
{
    if (!p) {
        *why = "params is NULL";
        return false;
    }
    if (p->L < 4 || p->L % 2 != 0 || p->L > MUCA_MAX_L) {
        *why = "L must be even with 4 <= L <= 128";
        return false;
    }
    if (!muca::sweep_supported(p->L)) {
        *why = "no sweep kernel is built for this L";
        return false;
    }
    if (p->walkers == 0) {
        *why = "walkers must be >= 1";
        return false;
    }
    if (p->walkers > (1u << 30)) {
        *why = "walkers must be <= 2^30";
        return false;
    }
    return true;
}

muca_host::Layout layout_for(const muca_params* p)
{
    muca_host::Layout l{};
    const size_t L = p->L, N = L * L;
    const size_t wpad = muca::padded_walkers(p->walkers);
    const size_t words = L * muca::words_per_row(p->L);
    size_t off = 0;
    l.spins_off = off;
    l.spins_bytes = words * wpad * sizeof(uint32_t);
    off = align_up(off + l.spins_bytes);
    l.energy_off = off;
    l.energy_bytes = wpad * sizeof(int32_t);
    off = align_up(off + l.energy_bytes);
    l.hist_off = off;
    l.hist_bytes = (N + 1) * sizeof(uint64_t);
    off = align_up(off + l.hist_bytes);
    l.table_off = off;
    l.table_bytes = (N + 1) * 4 * sizeof(uint64_t);
    off = align_up(off + l.table_bytes);
    l.total = off;
    return l;
}

// Message of the last failure with no instance to hold it (muca_create, the
// allocation-free production call): a fixed buffer, so that setting it never
// allocates.
thread_local char g_null_error[256];

}  // namespace

namespace muca_host {

void set_null_error(const char* msg)
{
    std::snprintf(g_null_error, sizeof g_null_error, "%s", msg);
}

}  // namespace muca_host

namespace {

int fail(muca_instance* h, int code, const std::string& msg)
{
    if (h)
        h->err = msg;
    else
        muca_host::set_null_error(msg.c_str());
    return code;
}

int device_fail(muca_instance* h, hipError_t e, const char* what)
{
    std::string msg = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    if (h)
        h->poisoned = true;
    return fail(h, MUCA_ERR_DEVICE, msg);
}

#define MUCA_HIP(h, call, what)                     \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess)                       \
            return device_fail((h), e_, (what));    \
    } while (0)

}  // namespace

namespace muca_host {

int finish_call(muca_instance* h, uint64_t therm, uint64_t recorded, bool update, double kernel_ms,
                uint32_t launches, uint32_t variant, muca_info* info)
{
    const uint32_t N = h->N;
    const uint64_t total = therm + recorded;
    h->position += total;
    const uint64_t* H = h->hist.data();
    uint64_t sum = 0;
    uint32_t visited = 0;
    for (uint32_t k = 0; k <= N; ++k) {
        sum += H[k];
        visited += H[k] > 0;
    }
    const uint64_t expect = (uint64_t)h->p.walkers * recorded;
    if (sum != expect) {
        h->poisoned = true;
        char buf[160];
        std::snprintf(buf, sizeof buf, "histogram sum %llu != walkers*recorded attempts %llu",
                      (unsigned long long)sum, (unsigned long long)expect);
        h->err = buf;
        return MUCA_ERR_DEVICE;
    }
    muca_info out{};
    out.attempts = (uint64_t)h->p.walkers * total;
    out.hist_sum = sum;
    out.sweep_counter = h->position / N;
    out.position = h->position;
    out.visited_bins = visited;
    out.flatness = flatness_of(N, H);
    out.kl_divergence = kl_of(N, H, h->reach_prev);
    out.width = (uint32_t)width_of(N, H);
    out.chebyshev = chebyshev_of(N, H);
    out.kernel_ms = kernel_ms;
    out.kernel_launches = launches;
    out.kernel_variant = variant;
    h->width_prev = (int)out.width;
    h->reach_prev = reach_of(N, H);
    if (update) {
        // Eq. 4, W <- W / H, in logarithmic form; empty bins keep omega.
        for (uint32_t k = 0; k <= N; ++k)
            if (H[k] > 0)
                h->omega[k] -= std::log((double)H[k]);
        ++h->iteration;
    }
    out.iteration = h->iteration;
    h->last = out;
    if (info)
        *info = out;
    return MUCA_OK;
}

}  // namespace muca_host

using namespace muca_host;

namespace {

int check_live(const muca_instance* h)
{
    if (!h)
        return MUCA_ERR_INVALID_ARG;
    if (h->poisoned)
        return MUCA_ERR_STATE;
    return MUCA_OK;
}

void release(muca_instance* h)
{
    if (!h)
        return;
    if (h->stream)
        (void)hipStreamSynchronize(h->stream);
    if (h->ev_start)
        (void)hipEventDestroy(h->ev_start);
    if (h->ev_stop)
        (void)hipEventDestroy(h->ev_stop);
    if (h->h_table4)
        (void)hipHostFree(h->h_table4);
    if (h->h_hist)
        (void)hipHostFree(h->h_hist);
    if (h->own_ws && h->ws)
        (void)hipFree(h->ws);
    if (h->own_stream && h->stream)
        (void)hipStreamDestroy(h->stream);
    delete h;
}

}  // namespace

namespace muca_host {

hipError_t enqueue_call(const CallTarget& t, const uint64_t* table5, const Segment* segs, size_t nsegs,
                        hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_stop, uint32_t* launches_out,
                        uint32_t* variant_out, const char** what)
{
    const uint32_t N = t.L * t.L;
    const size_t table_bytes = (size_t)(N + 1) * 4 * sizeof(uint64_t);
    // kernel choice: 5 two-wave pairs, 4 wide two-wave, 3 wide, 2 split,
    // 1 fast, 0 generic (all give the same bits)
    uint32_t variant = 0;
    if (!(t.flags & MUCA_FLAG_GENERIC_KERNEL) && muca::wide_sweep_supported(t.L) &&
        fast_table(N, table5, reinterpret_cast<uint32_t*>(t.h_table4), 8)) {
        // as for L <= 64: a second wave for the random numbers pays while every
        // workgroup is resident at once
        const bool two = !(t.flags & MUCA_FLAG_FAST_KERNEL) && muca::wide_split_supported(t.L) &&
                         muca::prefer_wide_split(t.L, t.wpad / muca::kWave, (uint32_t)t.cus);
        variant = two ? 4 : 3;
    } else if (!(t.flags & MUCA_FLAG_GENERIC_KERNEL) &&
               (muca::split_sweep_supported(t.L) || muca::fast_sweep_supported(t.L)) &&
               fast_table(N, table5, reinterpret_cast<uint32_t*>(t.h_table4), 5)) {
        // The split kernel gives each 64 walkers a second wave for the random
        // numbers; once its workgroups no longer all fit at once, or more than
        // two share a CU, the one-wave form wins.
        // Where one two-wave workgroup fills a CU and the blocks outnumber
        // the CUs, the pair form gives each CU two chains.
        const uint64_t blocks = t.wpad / muca::kWave;
        const bool forced_fast = (t.flags & MUCA_FLAG_FAST_KERNEL) != 0;
        const bool pair = !forced_fast && muca::prefer_pair(t.L, blocks, (uint32_t)t.cus);
        const bool want_fast = forced_fast || (!muca::prefer_split(t.L, blocks, (uint32_t)t.cus) &&
                                               muca::fast_sweep_supported(t.L));
        if (pair)
            variant = 5;
        else if (muca::split_sweep_supported(t.L) && !(want_fast && muca::fast_sweep_supported(t.L)))
            variant = 2;
        else
            variant = 1;
    }
    const bool fast = variant != 0;
    if (!fast)
        device_table(N, table5, t.h_table4);
    *variant_out = variant;
    *launches_out = 0;
#define MUCA_ENQ(call, msg)          \
    do {                             \
        hipError_t e_ = (call);      \
        if (e_ != hipSuccess) {      \
            *what = (msg);           \
            return e_;               \
        }                            \
    } while (0)
    MUCA_ENQ(hipMemcpyAsync(t.d_table, t.h_table4, table_bytes, hipMemcpyHostToDevice, stream),
             "threshold upload");
    MUCA_ENQ(muca::launch_fill_u64(t.d_hist, N + 1, stream), "histogram clear");

    uint32_t chunk = muca::max_sweeps_per_launch(t.L);
    const uint32_t cap = t.flags & MUCA_FLAG_SWEEPS_PER_LAUNCH_MASK;
    if (cap != 0 && cap < chunk)
        chunk = cap;
    uint32_t launches = 0;
    if (ev_start)
        MUCA_ENQ(hipEventRecord(ev_start, stream), "hipEventRecord");
    for (size_t i = 0; i < nsegs; ++i) {
        const Segment& g = segs[i];
        if (g.n == 0) {
            muca::RangeArgs a{};
            a.spins = t.d_spins;
            a.energy = t.d_energy;
            a.table = t.d_table;
            a.hist = t.d_hist;
            a.sweep = g.sweep0;
            a.L = t.L;
            a.wpad = t.wpad;
            a.walkers = t.walkers;
            a.seed = t.seed;
            a.site_begin = g.site_begin;
            a.site_end = g.site_end;
            a.rec_begin = g.rec_begin;
            a.table_stride = (variant == 3 || variant == 4) ? 8u : (fast ? 5u : 0u);
            MUCA_ENQ(muca::launch_sweep_range(a, stream), "partial sweep launch");
            ++launches;
            continue;
        }
        for (uint64_t s0 = 0; s0 < g.n; s0 += chunk) {
            const uint32_t n = (uint32_t)std::min<uint64_t>(g.n - s0, chunk);
            const uint32_t th = s0 >= g.therm ? 0u : (uint32_t)std::min<uint64_t>(g.therm - s0, n);
            if (fast) {
                muca::FastSweepArgs a{};
                a.spins = t.d_spins;
                a.energy = t.d_energy;
                a.table = reinterpret_cast<const uint32_t*>(t.d_table);
                a.hist = t.d_hist;
                a.sweep0 = g.sweep0 + s0;
                a.wpad = t.wpad;
                a.walkers = t.walkers;
                a.seed = t.seed;
                a.nsweeps = n;
                a.therm = th;
                MUCA_ENQ(variant == 5   ? muca::launch_pair_sweep(t.L, a, stream)
                         : variant == 4 ? muca::launch_wide_split_sweep(t.L, a, stream)
                         : variant == 3 ? muca::launch_wide_sweep(t.L, a, stream)
                         : variant == 2 ? muca::launch_split_sweep(t.L, a, stream)
                                        : muca::launch_fast_sweep(t.L, a, stream),
                         "sweep launch");
            } else {
                muca::SweepArgs a{};
                a.spins = t.d_spins;
                a.energy = t.d_energy;
                a.table = t.d_table;
                a.hist = t.d_hist;
                a.sweep0 = g.sweep0 + s0;
                a.wpad = t.wpad;
                a.walkers = t.walkers;
                a.seed = t.seed;
                a.nsweeps = n;
                a.therm = th;
                MUCA_ENQ(muca::launch_sweep(t.L, a, stream), "sweep launch");
            }
            ++launches;
        }
    }
    if (ev_stop)
        MUCA_ENQ(hipEventRecord(ev_stop, stream), "hipEventRecord");
#undef MUCA_ENQ
    *launches_out = launches;
    return hipSuccess;
}

}  // namespace muca_host

namespace {

// therm unrecorded, then `recorded` recorded attempts per walker, starting at
// the instance's position; H -> h->hist.
int run_attempts(muca_instance* h, uint64_t therm, uint64_t recorded, bool update, muca_info* info)
{
    int rc = check_live(h);
    if (rc != MUCA_OK)
        return rc;
    const uint32_t N = h->N;
    const uint64_t total = therm + recorded;
    if (total < therm)
        return fail(h, MUCA_ERR_OVERFLOW, "attempt count wraps");
    const long double attempts_ld = (long double)h->p.walkers * (long double)total;
    if (attempts_ld >= 18446744073709551615.0L)
        return fail(h, MUCA_ERR_OVERFLOW, "walkers * attempts exceeds 2^64");
    if (h->position + total < h->position)
        return fail(h, MUCA_ERR_OVERFLOW, "attempt position would wrap");

    std::vector<muca_host::Segment> segments;
    try {
        segments = muca_host::segments_of(N, h->position, therm, recorded);
    } catch (const std::bad_alloc&) {
        return fail(h, MUCA_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    compute_thresholds(N, h->omega.data(), h->table5.data());
    muca_host::CallTarget t{};
    t.L = h->L;
    t.wpad = h->wpad;
    t.walkers = h->p.walkers;
    t.seed = h->p.seed;
    t.flags = h->p.flags;
    t.cus = h->cus;
    t.d_spins = h->d_spins;
    t.d_energy = h->d_energy;
    t.d_hist = h->d_hist;
    t.d_table = h->d_table;
    t.h_table4 = h->h_table4;
    MUCA_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    uint32_t launches = 0, variant = 0;
    const char* what = "";
    hipError_t e = muca_host::enqueue_call(t, h->table5.data(), segments.data(), segments.size(), h->stream,
                                           h->ev_start, h->ev_stop, &launches, &variant, &what);
    if (e != hipSuccess)
        return device_fail(h, e, what);
    MUCA_HIP(h, hipMemcpyAsync(h->h_hist, h->d_hist, h->lay.hist_bytes, hipMemcpyDeviceToHost,
                               h->stream),
             "histogram download");
    MUCA_HIP(h, hipStreamSynchronize(h->stream), "sweep stream");
    float ms = 0.0f;
    if (launches)
        MUCA_HIP(h, hipEventElapsedTime(&ms, h->ev_start, h->ev_stop), "hipEventElapsedTime");

    std::memcpy(h->hist.data(), h->h_hist, h->lay.hist_bytes);
    return finish_call(h, therm, recorded, update, ms, launches, variant, info);
}

}  // namespace

extern "C" {

size_t muca_state_bytes(const muca_params* p)
{
    std::string why;
    if (!params_valid(p, &why))
        return 0;
    return layout_for(p).total;
}

int muca_create(const muca_params* p, void* hip_stream, void* device_workspace,
                size_t workspace_bytes, muca_instance** out)
{
    if (!out)
        return fail(nullptr, MUCA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!params_valid(p, &why))
        return fail(nullptr, MUCA_ERR_INVALID_ARG, why);
    muca_instance* h = new (std::nothrow) muca_instance();
    if (!h)
        return fail(nullptr, MUCA_ERR_OUT_OF_MEMORY, "host allocation failed");
    h->p = *p;
    h->L = p->L;
    h->N = p->L * p->L;
    h->wpr = muca::words_per_row(p->L);
    h->wpad = muca::padded_walkers(p->walkers);
    h->lay = layout_for(p);
    try {
        h->omega.assign(h->N + 1, 0.0);
        h->table5.assign((size_t)(h->N + 1) * 5, 0);
        h->hist.assign(h->N + 1, 0);
    } catch (...) {
        delete h;
        return fail(nullptr, MUCA_ERR_OUT_OF_MEMORY, "host allocation failed");
    }

    auto bail = [&](int code) {
        muca_host::set_null_error(h->err.c_str());
        release(h);
        return code;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        device_fail(h, e, "hipGetDevice");
        return bail(MUCA_ERR_DEVICE);
    }
    e = hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device);
    if (e != hipSuccess) {
        device_fail(h, e, "hipDeviceGetAttribute");
        return bail(MUCA_ERR_DEVICE);
    }
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreate(&h->stream);
        if (e != hipSuccess) {
            device_fail(h, e, "hipStreamCreate");
            return bail(MUCA_ERR_DEVICE);
        }
        h->own_stream = true;
    }
    if (device_workspace) {
        if (workspace_bytes < h->lay.total || ((uintptr_t)device_workspace % kAlign) != 0) {
            fail(h, MUCA_ERR_OUT_OF_MEMORY, "workspace too small or not 256-byte aligned");
            return bail(MUCA_ERR_OUT_OF_MEMORY);
        }
        h->ws = device_workspace;
    } else {
        e = hipMalloc(&h->ws, h->lay.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->ws = nullptr;
            fail(h, MUCA_ERR_OUT_OF_MEMORY, "device allocation of the instance state failed");
            return bail(MUCA_ERR_OUT_OF_MEMORY);
        }
        h->own_ws = true;
    }
    char* base = (char*)h->ws;
    h->d_spins = (uint32_t*)(base + h->lay.spins_off);
    h->d_energy = (int32_t*)(base + h->lay.energy_off);
    h->d_hist = (unsigned long long*)(base + h->lay.hist_off);
    h->d_table = (uint64_t*)(base + h->lay.table_off);
    if (hipHostMalloc((void**)&h->h_table4, h->lay.table_bytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h->h_hist, h->lay.hist_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        fail(h, MUCA_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
        return bail(MUCA_ERR_OUT_OF_MEMORY);
    }
    if ((e = hipEventCreate(&h->ev_start)) != hipSuccess ||
        (e = hipEventCreate(&h->ev_stop)) != hipSuccess) {
        device_fail(h, e, "hipEventCreate");
        return bail(MUCA_ERR_DEVICE);
    }
    muca::InitArgs ia{};
    ia.spins = h->d_spins;
    ia.energy = h->d_energy;
    ia.L = h->L;
    ia.wpad = h->wpad;
    ia.seed = p->seed;
    if ((e = muca::launch_init(ia, h->stream)) != hipSuccess) {
        device_fail(h, e, "init launch");
        return bail(MUCA_ERR_DEVICE);
    }
    if ((e = muca::launch_fill_u64(h->d_hist, h->N + 1, h->stream)) != hipSuccess) {
        device_fail(h, e, "histogram clear");
        return bail(MUCA_ERR_DEVICE);
    }
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) {
        device_fail(h, e, "init stream");
        return bail(MUCA_ERR_DEVICE);
    }
    compute_thresholds(h->N, h->omega.data(), h->table5.data());
    *out = h;
    return MUCA_OK;
}

int muca_destroy(muca_instance* h)
{
    release(h);
    return MUCA_OK;
}

int muca_iterate(muca_instance* h, uint32_t therm_sweeps, uint32_t sweeps, muca_info* info)
{
    if (!h)
        return MUCA_ERR_INVALID_ARG;
    return run_attempts(h, (uint64_t)therm_sweeps * h->N, (uint64_t)sweeps * h->N, true, info);
}

int muca_production(muca_instance* h, uint32_t therm_sweeps, uint32_t sweeps, muca_info* info)
{
    if (!h)
        return MUCA_ERR_INVALID_ARG;
    return run_attempts(h, (uint64_t)therm_sweeps * h->N, (uint64_t)sweeps * h->N, false, info);
}

int muca_iterate_attempts(muca_instance* h, uint64_t therm_attempts, uint64_t attempts, muca_info* info)
{
    return run_attempts(h, therm_attempts, attempts, true, info);
}

int muca_production_attempts(muca_instance* h, uint64_t therm_attempts, uint64_t attempts,
                             muca_info* info)
{
    return run_attempts(h, therm_attempts, attempts, false, info);
}

int muca_run_schedule(muca_instance* h, const muca_schedule* sc, muca_schedule_step* steps,
                      uint32_t max_steps, uint32_t* iterations)
{
    if (iterations)
        *iterations = 0;
    if (int rc = check_live(h))
        return rc;
    if (!sc || !(sc->z > 0.0) || !(sc->growth >= 1.0) || sc->max_iterations == 0 ||
        sc->stop_rule > MUCA_STOP_CHEBYSHEV)
        return fail(h, MUCA_ERR_INVALID_ARG, "schedule needs z > 0, growth >= 1, max_iterations > 0, a known stop rule");
    const bool chebyshev = sc->stop_rule == MUCA_STOP_CHEBYSHEV;
    const double stop_below = chebyshev ? sc->dc_flat : sc->dk_flat;
    if (!(stop_below > 0.0))
        return fail(h, MUCA_ERR_INVALID_ARG, "the stop rule's threshold must be > 0");
    if (steps == nullptr && max_steps != 0)
        return fail(h, MUCA_ERR_INVALID_ARG, "steps is NULL");
    const uint32_t N = h->N;
    const double walkers = (double)h->p.walkers;
    double x = 0.0;
    bool full = false;
    for (uint32_t it = 0; it < sc->max_iterations; ++it) {
        // Sec. 3: w = max(w', w_min), w' the range the previous iteration covered
        const uint32_t w = std::max<uint32_t>((uint32_t)h->width_prev, sc->w_min);
        if (full) {
            x = x * sc->growth;
        } else {
            x = 6.0 * std::pow((double)w, sc->z) / walkers;  // Eq. 7
            full = w == N + 1;
        }
        if (!(x < 1.8e19))
            return fail(h, MUCA_ERR_OVERFLOW, "update count of the schedule passes 2^64");
        const uint64_t updates = (uint64_t)std::floor(x) + 1;
        const uint64_t therm = (uint64_t)sc->f_therm * w;
        muca_info info{};
        if (int rc = run_attempts(h, therm, updates, true, &info))
            return rc;
        if (iterations)
            *iterations = it + 1;
        if (it < max_steps) {
            muca_schedule_step st{};
            st.therm_attempts = therm;
            st.update_attempts = updates;
            st.kl_divergence = info.kl_divergence;
            st.chebyshev = info.chebyshev;
            st.flatness = info.flatness;
            st.kernel_ms = info.kernel_ms;
            st.width = w;
            st.covered = info.width;
            steps[it] = st;
        }
        if (full && (chebyshev ? info.chebyshev : info.kl_divergence) < stop_below)
            return MUCA_OK;
    }
    return fail(h, MUCA_ERR_NOT_CONVERGED, "the schedule reached max_iterations");
}

int muca_histogram(const muca_instance* h, uint64_t* out, size_t n_bins)
{
    int rc = check_live(h);
    if (rc != MUCA_OK)
        return rc;
    if (!out || n_bins != (size_t)h->N + 1)
        return fail(const_cast<muca_instance*>(h), MUCA_ERR_INVALID_ARG, "n_bins must be L*L+1");
    std::memcpy(out, h->hist.data(), n_bins * sizeof(uint64_t));
    return MUCA_OK;
}

int muca_log_weights(const muca_instance* h, double* out, size_t n_bins)
{
    int rc = check_live(h);
    if (rc != MUCA_OK)
        return rc;
    if (!out || n_bins != (size_t)h->N + 1)
        return fail(const_cast<muca_instance*>(h), MUCA_ERR_INVALID_ARG, "n_bins must be L*L+1");
    std::memcpy(out, h->omega.data(), n_bins * sizeof(double));
    return MUCA_OK;
}

int muca_set_log_weights(muca_instance* h, const double* in, size_t n_bins)
{
    int rc = check_live(h);
    if (rc != MUCA_OK)
        return rc;
    if (!in || n_bins != (size_t)h->N + 1)
        return fail(h, MUCA_ERR_INVALID_ARG, "n_bins must be L*L+1");
    for (size_t k = 0; k < n_bins; ++k)
        if (!std::isfinite(in[k]))
            return fail(h, MUCA_ERR_INVALID_ARG, "log weights must be finite");
    std::memcpy(h->omega.data(), in, n_bins * sizeof(double));
    return MUCA_OK;
}

int muca_thresholds(const muca_instance* h, uint64_t* out, size_t n)
{
    int rc = check_live(h);
    if (rc != MUCA_OK)
        return rc;
    if (!out || n != ((size_t)h->N + 1) * 5)
        return fail(const_cast<muca_instance*>(h), MUCA_ERR_INVALID_ARG, "n must be 5*(L*L+1)");
    std::memcpy(out, h->table5.data(), n * sizeof(uint64_t));
    return MUCA_OK;
}

int muca_energies(const muca_instance* h, int32_t* out, size_t walkers)
{
    int rc = check_live(h);
    if (rc != MUCA_OK)
        return rc;
    muca_instance* m = const_cast<muca_instance*>(h);
    if (!out || walkers != h->p.walkers)
        return fail(m, MUCA_ERR_INVALID_ARG, "walkers must equal the instance's walker count");
    MUCA_HIP(m, hipSetDevice(h->device), "hipSetDevice");
    MUCA_HIP(m, hipMemcpyAsync(out, h->d_energy, walkers * sizeof(int32_t), hipMemcpyDeviceToHost,
                               h->stream),
             "energy download");
    MUCA_HIP(m, hipStreamSynchronize(h->stream), "energy download");
    return MUCA_OK;
}

int muca_spins(const muca_instance* h, int8_t* out, size_t n)
{
    int rc = check_live(h);
    if (rc != MUCA_OK)
        return rc;
    muca_instance* m = const_cast<muca_instance*>(h);
    const size_t N = h->N;
    if (!out || n != (size_t)h->p.walkers * N)
        return fail(m, MUCA_ERR_INVALID_ARG, "n must be walkers*L*L");
    std::vector<uint32_t> words;
    try {
        words.resize((size_t)h->L * h->wpr * h->wpad);
    } catch (...) {
        return fail(m, MUCA_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    MUCA_HIP(m, hipSetDevice(h->device), "hipSetDevice");
    MUCA_HIP(m, hipMemcpyAsync(words.data(), h->d_spins, words.size() * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, h->stream),
             "spin download");
    MUCA_HIP(m, hipStreamSynchronize(h->stream), "spin download");
    const uint32_t L = h->L, wpr = h->wpr;
    for (size_t w = 0; w < h->p.walkers; ++w)
        for (uint32_t y = 0; y < L; ++y)
            for (uint32_t x = 0; x < L; ++x) {
                const uint32_t word = words[(size_t)(y * wpr + x / 32) * h->wpad + w];
                out[w * N + (size_t)y * L + x] = ((word >> (x % 32)) & 1u) ? 1 : -1;
            }
    return MUCA_OK;
}

namespace {

// Checkpoint layout: a header, then omega[N+1] (double), hist[N+1] (uint64),
// energies[wpad] (int32) and the lattice words[L * wpr * wpad] (uint32) in the
// device layout (padding walkers included, so that a restored instance
// continues bit for bit).
struct CheckpointHeader {
    uint32_t magic;    // 'MUCK'
    uint32_t version;  // 1
    uint32_t L, walkers, seed, wpad;
    uint64_t position;
    uint32_t iteration;
    int32_t width_prev, reach_prev;
    uint32_t reserved;
};
constexpr uint32_t kCheckpointMagic = 0x4b43554du;

size_t checkpoint_bytes(const muca_instance* h)
{
    const size_t N1 = (size_t)h->N + 1;
    return sizeof(CheckpointHeader) + N1 * sizeof(double) + N1 * sizeof(uint64_t) +
           (size_t)h->wpad * sizeof(int32_t) + (size_t)h->L * h->wpr * h->wpad * sizeof(uint32_t);
}

}  // namespace

size_t muca_checkpoint_bytes(const muca_instance* h)
{
    return h ? checkpoint_bytes(h) : 0;
}

int muca_checkpoint(const muca_instance* h, void* out, size_t n)
{
    int rc = check_live(h);
    if (rc != MUCA_OK)
        return rc;
    muca_instance* m = const_cast<muca_instance*>(h);
    if (!out || n != checkpoint_bytes(h))
        return fail(m, MUCA_ERR_INVALID_ARG, "n must be muca_checkpoint_bytes(h)");
    const size_t N1 = (size_t)h->N + 1;
    char* p = static_cast<char*>(out);
    CheckpointHeader hd{};
    hd.magic = kCheckpointMagic;
    hd.version = 1;
    hd.L = h->L;
    hd.walkers = h->p.walkers;
    hd.seed = h->p.seed;
    hd.wpad = h->wpad;
    hd.position = h->position;
    hd.iteration = h->iteration;
    hd.width_prev = h->width_prev;
    hd.reach_prev = h->reach_prev;
    std::memcpy(p, &hd, sizeof hd);
    p += sizeof hd;
    std::memcpy(p, h->omega.data(), N1 * sizeof(double));
    p += N1 * sizeof(double);
    std::memcpy(p, h->hist.data(), N1 * sizeof(uint64_t));
    p += N1 * sizeof(uint64_t);
    MUCA_HIP(m, hipSetDevice(h->device), "hipSetDevice");
    MUCA_HIP(m, hipMemcpyAsync(p, h->d_energy, (size_t)h->wpad * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream),
             "energy download");
    p += (size_t)h->wpad * sizeof(int32_t);
    MUCA_HIP(m, hipMemcpyAsync(p, h->d_spins, (size_t)h->L * h->wpr * h->wpad * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, h->stream),
             "spin download");
    MUCA_HIP(m, hipStreamSynchronize(h->stream), "checkpoint download");
    return MUCA_OK;
}

int muca_restore(muca_instance* h, const void* in, size_t n)
{
    int rc = check_live(h);
    if (rc != MUCA_OK)
        return rc;
    if (!in || n != checkpoint_bytes(h))
        return fail(h, MUCA_ERR_INVALID_ARG, "n must be muca_checkpoint_bytes(h)");
    const char* p = static_cast<const char*>(in);
    CheckpointHeader hd;
    std::memcpy(&hd, p, sizeof hd);
    if (hd.magic != kCheckpointMagic || hd.version != 1)
        return fail(h, MUCA_ERR_INVALID_ARG, "not a checkpoint of this library");
    if (hd.L != h->L || hd.walkers != h->p.walkers || hd.seed != h->p.seed || hd.wpad != h->wpad)
        return fail(h, MUCA_ERR_INVALID_ARG, "checkpoint of an instance with other L, walkers or seed");
    const size_t N1 = (size_t)h->N + 1;
    const double* om = reinterpret_cast<const double*>(p + sizeof hd);
    for (size_t k = 0; k < N1; ++k) {
        double v;
        std::memcpy(&v, om + k, sizeof v);
        if (!std::isfinite(v))
            return fail(h, MUCA_ERR_INVALID_ARG, "checkpoint holds a non-finite log weight");
    }
    const char* pe = p + sizeof hd + N1 * (sizeof(double) + sizeof(uint64_t));
    const int32_t lo = -2 * (int32_t)h->N, hi = 2 * (int32_t)h->N;
    for (size_t w = 0; w < h->wpad; ++w) {
        int32_t e;
        std::memcpy(&e, pe + w * sizeof(int32_t), sizeof e);
        if (e < lo || e > hi || (e - lo) % 4 != 0)
            return fail(h, MUCA_ERR_INVALID_ARG, "checkpoint holds an impossible energy");
    }
    MUCA_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    MUCA_HIP(h, hipMemcpyAsync(h->d_energy, pe, (size_t)h->wpad * sizeof(int32_t), hipMemcpyHostToDevice, h->stream),
             "energy upload");
    MUCA_HIP(h, hipMemcpyAsync(h->d_spins, pe + (size_t)h->wpad * sizeof(int32_t),
                               (size_t)h->L * h->wpr * h->wpad * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream),
             "spin upload");
    MUCA_HIP(h, hipStreamSynchronize(h->stream), "checkpoint upload");
    std::memcpy(h->omega.data(), p + sizeof hd, N1 * sizeof(double));
    std::memcpy(h->hist.data(), p + sizeof hd + N1 * sizeof(double), N1 * sizeof(uint64_t));
    h->position = hd.position;
    h->iteration = hd.iteration;
    h->width_prev = hd.width_prev;
    h->reach_prev = hd.reach_prev;
    return MUCA_OK;
}

int muca_log_dos(const muca_instance* h, int normalization, double* out, size_t n)
{
    int rc = check_live(h);
    if (rc != MUCA_OK)
        return rc;
    muca_instance* m = const_cast<muca_instance*>(h);
    const uint32_t N = h->N;
    if (!out || n != (size_t)N + 1 || (normalization != 0 && normalization != 1))
        return fail(m, MUCA_ERR_INVALID_ARG, "n must be L*L+1 and normalization 0 or 1");
    switch (log_dos_of(N, h->hist.data(), h->omega.data(), normalization, out)) {
    case 1:
        return fail(m, MUCA_ERR_NOT_CONVERGED, "ground-state bin is empty");
    case 2:
        return fail(m, MUCA_ERR_NOT_CONVERGED, "histogram is empty");
    default:
        return MUCA_OK;
    }
}

int muca_last_info(const muca_instance* h, muca_info* out)
{
    if (!h || !out)
        return MUCA_ERR_INVALID_ARG;
    *out = h->last;
    return h->poisoned ? MUCA_ERR_STATE : MUCA_OK;
}

const char* muca_last_error(const muca_instance* h)
{
    return h ? h->err.c_str() : g_null_error;
}

}  // extern "C"
