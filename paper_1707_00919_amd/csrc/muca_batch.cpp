// muca_batch.cpp -- batched rounds over many independent instances
// (include/muca.h, muca_batch_*).
//
// Each member is its own parallel multicanonical run (Sec. 2.2: a walker
// population with its own weights and histogram).  A small instance alone
// fills a few compute units; a round of the batch sweeps all members together:
//   host   thresholds of every running member into one pinned staging buffer,
//          together with the per-member kernel arguments and the list of
//          workgroups (member, 64-walker block);
//   device one upload, one clear of the batch histogram buffer, one launch per
//          (L, kernel form) group -- the groups on streams of their own so that
//          they run side by side -- and one download of all histograms;
//   host   per member the same finish as a single call (sum check, statistics,
//          Eq. 4 for iterations).
// The device work of a round can be captured in a HIP graph and replayed while
// the round's shape stays the same.  Kernels, arguments and random-number
// labels per walker are those of a single call, so every member's results are
// bit-identical to running it alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "muca.h"
#include "muca_device.h"
#include "muca_internal.h"

using namespace muca_host;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

thread_local std::string g_batch_error;

// kernel forms, as in muca_info::kernel_variant
constexpr uint32_t kGeneric = muca_host::kFormGeneric, kFast = muca_host::kFormFast, kSplit = muca_host::kFormSplit,
                   kWide = muca_host::kFormWide, kWideSplit = muca_host::kFormWideSplit, kPair = muca_host::kFormPair;

bool two_wave_form(uint32_t form) { return form == kSplit || form == kPair || form == kWideSplit; }

// A round's launches are issued longest chains first -- the two-wave groups,
// then the others, each kind by its longest chain -- and, in rounds where
// placement can hold a workgroup back, each one after the first behind a wait
// of this many microseconds more than the one before, long enough for the
// earlier launches to have placed their workgroups (muca_order.hip); from the
// ninth launch on the wait stays at its eighth step (the shortest chains come
// last, and their order among themselves hardly matters).
constexpr uint32_t kDispatchDelayUs = 30;
constexpr uint32_t kDispatchSteps = 8;

struct Group {
    uint32_t L = 0;
    uint32_t form = kGeneric;
    uint32_t waves = 1;       // waves of 64 walkers per workgroup (one-wave form)
    uint32_t first_item = 0;  // index into the items array
    uint32_t nitems = 0;
    uint64_t chain = 0;       // attempts of the group's longest walker chain
};

// Launch shapes of a round, for members that can run the LDS-record kernels:
// the two-wave form for all (at L = 48-64 in pairs, two chains per table,
// where one workgroup per chain does not fit); the one-wave form with its
// default wave groups, or with four waves (256 walkers) sharing each table;
// the mixed shape -- the two-wave form for the members with the longest
// chains per round, as many as fit on the device at once, the one-wave form
// for the others; the mixed-longest shape -- the two-wave form only for the
// members whose chain is the round's longest, so that the shorter chains start
// at once on the CUs those leave, instead of waiting for a CU that the
// two-wave workgroups of the next-longest hold; and the histogram-merge
// cadence -- the round's default shape with its sweeps cut into two launches,
// so that every workgroup's LDS counters are merged into the global histogram
// twice per round instead of once.  A round whose two-wave workgroups all fit
// runs the two-wave form; the others run the mixed-longest shape, or with the
// autotuner the fastest of the last five, timed on five rounds and timed again
// once the rounds' walkers have halved since.
constexpr int kChoices = 6;
constexpr int kTwoWave = muca_host::kShapeTwoWave, kOneWaveDefault = muca_host::kShapeOneWave,
              kOneWaveFour = muca_host::kShapeOneWaveFour, kTwoMerges = 3, kMixed = muca_host::kShapeMixed,
              kMixedLongest = muca_host::kShapeMixedLongest;
constexpr int kTuned[5] = {kMixedLongest, kMixed, kOneWaveDefault, kOneWaveFour, kTwoMerges};
constexpr uint32_t kNumTuned = sizeof(kTuned) / sizeof(kTuned[0]);

}  // namespace

struct muca_batch {
    std::vector<muca_instance*> m;
    uint32_t flags = 0;
    int device = 0;
    int cus = 256;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<hipStream_t> gstreams;  // one per concurrently running group
    std::vector<hipEvent_t> gevents;
    hipEvent_t ev_fork = nullptr, ev_start = nullptr, ev_stop = nullptr;
    // staging: [fast args][generic args][items][tables], pinned and on device
    size_t off_fargs = 0, off_gargs = 0, off_items = 0, off_tables = 0, stage_bytes = 0;
    std::vector<size_t> table_off, hist_off;
    void* h_stage = nullptr;
    void* d_stage = nullptr;
    unsigned long long* d_hist = nullptr;
    uint64_t* h_hist = nullptr;
    size_t hist_words = 0;
    size_t stage_cap = 0, hist_cap = 0;  // allocated sizes (bytes, words)
    // graph of the last round's device work
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string graph_key;
    hipEvent_t ev_done = nullptr;  // end of a submitted round (histograms on the host)
    // the submitted round, until muca_batch_finish
    bool pending = false;
    std::vector<uint32_t> mode, therm, sweeps, form;
    std::vector<uint64_t> total;
    uint32_t launches = 0;
    // with MUCA_BATCH_GRAPH the host half of a round runs inside the graph, as
    // a host node after the histogram download; its results wait here
    bool host_in_graph = false;
    // the submitted round's launches start staggered (crowded or paired rounds)
    bool stagger = false;
    std::vector<muca_info> round_infos;
    int host_rc = MUCA_OK;
    std::string host_err;
    // autotuner: attempts/ms of the shapes timed so far (rounds whose
    // two-wave workgroups do not all fit)
    uint32_t round = 0;
    double tuned_rate[kChoices] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int tuned_form = -1;
    uint32_t tune_step = 0;        // shapes timed since the last (re)start
    uint64_t tuned_walkers = 0;    // walkers of the round the choice was made on
    bool tuning = false;           // the submitted round is timed for the autotuner
    uint64_t round_walkers = 0;    // walkers of the submitted round
    int choice = kTwoWave;  // of the submitted round
    std::string err;
};

namespace {

int bfail(muca_batch* b, int code, const std::string& msg)
{
    if (b)
        b->err = msg;
    else
        g_batch_error = msg;
    return code;
}

#define BATCH_HIP(b, call, what)                                                             \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return bfail((b), MUCA_ERR_DEVICE,                                             \
                         std::string(what) + ": " + hipGetErrorName(e_) + " (" +           \
                             hipGetErrorString(e_) + ")");                                 \
    } while (0)

void drop_graph(muca_batch* b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_key.clear();
}

void release(muca_batch* b)
{
    if (!b)
        return;
    if (b->stream)
        (void)hipStreamSynchronize(b->stream);
    for (hipStream_t s : b->gstreams)
        (void)hipStreamSynchronize(s);
    drop_graph(b);
    for (hipStream_t s : b->gstreams)
        (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->gevents)
        (void)hipEventDestroy(e);
    if (b->ev_fork)
        (void)hipEventDestroy(b->ev_fork);
    if (b->ev_start)
        (void)hipEventDestroy(b->ev_start);
    if (b->ev_stop)
        (void)hipEventDestroy(b->ev_stop);
    if (b->ev_done)
        (void)hipEventDestroy(b->ev_done);
    if (b->h_stage)
        (void)hipHostFree(b->h_stage);
    if (b->h_hist)
        (void)hipHostFree(b->h_hist);
    if (b->d_stage)
        (void)hipFree(b->d_stage);
    if (b->d_hist)
        (void)hipFree(b->d_hist);
    if (b->own_stream && b->stream)
        (void)hipStreamDestroy(b->stream);
    delete b;
}

int ensure_group_streams(muca_batch* b, size_t n)
{
    while (b->gstreams.size() < n) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        BATCH_HIP(b, hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
        b->gstreams.push_back(s);
        BATCH_HIP(b, hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
        b->gevents.push_back(e);
    }
    return MUCA_OK;
}

// The device work of one launch round (enqueued on b->stream, or recorded
// into a graph when the stream is capturing).
int enqueue_round(muca_batch* b, size_t stage_used, const std::vector<Group>& groups)
{
    BATCH_HIP(b, hipMemcpyAsync(b->d_stage, b->h_stage, stage_used, hipMemcpyHostToDevice, b->stream),
              "batch upload");
    BATCH_HIP(b, hipEventRecord(b->ev_fork, b->stream), "hipEventRecord");
    char* ds = static_cast<char*>(b->d_stage);
    const auto* fargs = reinterpret_cast<const muca::FastSweepArgs*>(ds + b->off_fargs);
    const auto* gargs = reinterpret_cast<const muca::SweepArgs*>(ds + b->off_gargs);
    const auto* items = reinterpret_cast<const muca::BatchItem*>(ds + b->off_items);
    // groups come in dispatch order (muca_batch_submit): in a crowded or
    // paired round each after the first waits a little longer than the one
    // before
    for (size_t g = 0; g < groups.size(); ++g) {
        const Group& G = groups[g];
        hipStream_t s = b->gstreams[g];
        BATCH_HIP(b, hipStreamWaitEvent(s, b->ev_fork, 0), "hipStreamWaitEvent");
        if (g > 0 && b->stagger)
            BATCH_HIP(b, muca::launch_dispatch_delay((uint32_t)std::min<size_t>(g, kDispatchSteps) * kDispatchDelayUs, s),
                      "dispatch delay");
        hipError_t e;
        if (G.form == kSplit)
            e = muca::launch_split_batch(G.L, fargs, items + G.first_item, G.nitems, s);
        else if (G.form == kPair)
            e = muca::launch_pair_batch(G.L, fargs, items + G.first_item, G.nitems, s);
        else if (G.form == kWideSplit)
            e = muca::launch_wide_split_batch(G.L, fargs, items + G.first_item, G.nitems, s);
        else if (G.form == kWide)
            e = muca::launch_wide_batch(G.L, fargs, items + G.first_item, G.nitems, s);
        else if (G.form == kFast)
            e = muca::launch_fast_batch(G.L, G.waves, fargs, items + G.first_item, G.nitems, s);
        else
            e = muca::launch_sweep_batch(G.L, gargs, items + G.first_item, G.nitems, s);
        BATCH_HIP(b, e, "batched sweep launch");
        BATCH_HIP(b, hipEventRecord(b->gevents[g], s), "hipEventRecord");
        BATCH_HIP(b, hipStreamWaitEvent(b->stream, b->gevents[g], 0), "hipStreamWaitEvent");
    }
    return MUCA_OK;
}

// The host half of a round for every member that ran: histogram into the
// member, the same finish as a single call (sum check, statistics, Eq. 4).
int finish_members(muca_batch* b, double ms, std::vector<muca_info>& out, std::string* err)
{
    int result = MUCA_OK;
    out.assign(b->m.size(), muca_info{});
    for (size_t i = 0; i < b->m.size(); ++i) {
        if (b->mode[i] == MUCA_BATCH_SKIP)
            continue;
        muca_instance* h = b->m[i];
        std::memcpy(h->hist.data(), b->h_hist + b->hist_off[i], ((size_t)h->N + 1) * sizeof(uint64_t));
        const int rc = finish_call(h, (uint64_t)b->therm[i] * h->N, (uint64_t)b->sweeps[i] * h->N,
                                   b->mode[i] == MUCA_BATCH_ITERATE, ms, b->launches, b->form[i], &out[i]);
        if (rc != MUCA_OK && result == MUCA_OK) {
            result = rc;
            *err = "member " + std::to_string(i) + ": " + h->err;
        }
    }
    return result;
}

// Host node of a captured round.  It runs on a runtime thread once the
// histograms are on the host; it calls no HIP function.
void host_finish_node(void* arg)
{
    muca_batch* b = static_cast<muca_batch*>(arg);
    b->host_err.clear();
    b->host_rc = finish_members(b, 0.0, b->round_infos, &b->host_err);
}

}  // namespace

extern "C" {

int muca_batch_create(muca_instance* const* members, uint32_t count, void* hip_stream,
                      uint32_t flags, muca_batch** out)
{
    if (!out)
        return bfail(nullptr, MUCA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (flags & ~(uint32_t)(MUCA_BATCH_GRAPH | MUCA_BATCH_AUTOTUNE))
        return bfail(nullptr, MUCA_ERR_INVALID_ARG, "unknown batch flag");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return bfail(nullptr, MUCA_ERR_DEVICE, "hipGetDevice failed");
    muca_batch* b = new (std::nothrow) muca_batch();
    if (!b)
        return bfail(nullptr, MUCA_ERR_OUT_OF_MEMORY, "host allocation failed");
    auto bail = [&](int code) {
        g_batch_error = b->err;
        release(b);
        return code;
    };
    b->flags = flags;
    b->device = dev;
    if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        bfail(b, MUCA_ERR_DEVICE, "hipDeviceGetAttribute failed");
        return bail(MUCA_ERR_DEVICE);
    }
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&b->stream) != hipSuccess) {
            bfail(b, MUCA_ERR_DEVICE, "hipStreamCreate failed");
            return bail(MUCA_ERR_DEVICE);
        }
        b->own_stream = true;
    }
    if (hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&b->ev_start) != hipSuccess || hipEventCreate(&b->ev_stop) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming) != hipSuccess) {
        bfail(b, MUCA_ERR_DEVICE, "hipEventCreate failed");
        return bail(MUCA_ERR_DEVICE);
    }
    if (int rc = muca_batch_set_members(b, members, count))
        return bail(rc);
    *out = b;
    return MUCA_OK;
}

int muca_batch_set_members(muca_batch* b, muca_instance* const* members, uint32_t count)
{
    if (!b)
        return MUCA_ERR_INVALID_ARG;
    if (b->pending)
        return bfail(b, MUCA_ERR_STATE, "a submitted round has not been finished");
    if (!members || count == 0)
        return bfail(b, MUCA_ERR_INVALID_ARG, "a batch needs at least one member");
    for (uint32_t i = 0; i < count; ++i) {
        if (!members[i])
            return bfail(b, MUCA_ERR_INVALID_ARG, "NULL member");
        if (members[i]->poisoned)
            return bfail(b, MUCA_ERR_STATE, "a member is poisoned");
        if (members[i]->device != b->device)
            return bfail(b, MUCA_ERR_INVALID_ARG, "members must live on the batch's device");
    }
    {
        std::vector<const muca_instance*> sorted(members, members + count);
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return bfail(b, MUCA_ERR_INVALID_ARG, "a member appears twice");
    }
    // staging layout
    size_t total_blocks = 0, tables = 0, hist = 0;
    std::vector<size_t> table_off(count), hist_off(count);
    for (uint32_t i = 0; i < count; ++i) {
        const muca_instance* h = members[i];
        total_blocks += h->wpad / muca::kWave;
        table_off[i] = tables;
        tables += align_up(h->lay.table_bytes);
        hist_off[i] = hist;
        hist += (size_t)h->N + 1;
    }
    const size_t off_gargs = align_up(count * sizeof(muca::FastSweepArgs));
    const size_t off_items = align_up(off_gargs + count * sizeof(muca::SweepArgs));
    const size_t off_tables = align_up(off_items + total_blocks * sizeof(muca::BatchItem));
    const size_t stage_bytes = off_tables + tables;
    // buffers grow with headroom and are kept while a new member set fits,
    // so that a changing membership does not free device memory each time
    if (stage_bytes > b->stage_cap || hist > b->hist_cap) {
        if (b->stream)
            (void)hipStreamSynchronize(b->stream);
        if (b->h_stage)
            (void)hipHostFree(b->h_stage);
        if (b->h_hist)
            (void)hipHostFree(b->h_hist);
        if (b->d_stage)
            (void)hipFree(b->d_stage);
        if (b->d_hist)
            (void)hipFree(b->d_hist);
        b->h_stage = b->d_stage = nullptr;
        b->h_hist = nullptr;
        b->d_hist = nullptr;
        b->stage_cap = b->hist_cap = 0;
        const size_t scap = std::max(stage_bytes, stage_bytes + stage_bytes / 2);
        const size_t hcap = std::max(hist, hist + hist / 2);
        if (hipHostMalloc(&b->h_stage, scap, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&b->h_hist, hcap * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess ||
            hipMalloc(&b->d_stage, scap) != hipSuccess ||
            hipMalloc((void**)&b->d_hist, hcap * sizeof(uint64_t)) != hipSuccess) {
            (void)hipGetLastError();
            return bfail(b, MUCA_ERR_OUT_OF_MEMORY, "batch staging allocation failed");
        }
        std::memset(b->h_stage, 0, scap);
        b->stage_cap = scap;
        b->hist_cap = hcap;
    }
    try {
        b->m.assign(members, members + count);
        b->table_off = std::move(table_off);
        b->hist_off = std::move(hist_off);
        b->mode.assign(count, MUCA_BATCH_SKIP);
        b->therm.assign(count, 0);
        b->sweeps.assign(count, 0);
        b->form.assign(count, kGeneric);
        b->total.assign(count, 0);
    } catch (...) {
        return bfail(b, MUCA_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    b->off_fargs = 0;
    b->off_gargs = off_gargs;
    b->off_items = off_items;
    b->off_tables = off_tables;
    b->stage_bytes = stage_bytes;
    b->hist_words = hist;
    drop_graph(b);
    return MUCA_OK;
}

int muca_batch_destroy(muca_batch* b)
{
    release(b);
    return MUCA_OK;
}

const char* muca_batch_last_error(const muca_batch* b)
{
    return b ? b->err.c_str() : g_batch_error.c_str();
}

namespace {

// Poisons the members of the submitted round after a device failure: their
// lattices may have been swept while their host state was not advanced.
int poison_round(muca_batch* b, const std::string& why)
{
    for (size_t i = 0; i < b->m.size(); ++i)
        if (b->mode[i] != MUCA_BATCH_SKIP) {
            b->m[i]->poisoned = true;
            b->m[i]->err = "batched round failed: " + why;
        }
    b->pending = false;
    return MUCA_ERR_DEVICE;
}

}  // namespace

static int muca_batch_submit_impl(muca_batch* b, const uint32_t* mode, const uint32_t* therm,
                                  const uint32_t* sweeps)
{
    if (!b)
        return MUCA_ERR_INVALID_ARG;
    if (b->pending)
        return bfail(b, MUCA_ERR_STATE, "a submitted round has not been finished");
    if (!mode || !therm || !sweeps)
        return bfail(b, MUCA_ERR_INVALID_ARG, "mode, therm and sweeps are required");
    const uint32_t count = (uint32_t)b->m.size();
    BATCH_HIP(b, hipSetDevice(b->device), "hipSetDevice");

    // -- host: validate, thresholds, kernel form per member
    uint32_t active = 0, chunk = 0x7fffffffu;
    size_t active_blocks = 0;
    for (uint32_t i = 0; i < count; ++i) {
        if (mode[i] == MUCA_BATCH_SKIP)
            continue;
        if (mode[i] != MUCA_BATCH_ITERATE && mode[i] != MUCA_BATCH_PRODUCTION)
            return bfail(b, MUCA_ERR_INVALID_ARG, "mode must be SKIP, ITERATE or PRODUCTION");
        const muca_instance* h = b->m[i];
        if (h->poisoned)
            return bfail(b, MUCA_ERR_STATE, "member " + std::to_string(i) + " is poisoned");
        if (h->position % h->N != 0)
            return bfail(b, MUCA_ERR_INVALID_ARG,
                         "member " + std::to_string(i) + " stopped inside a sweep; batched rounds run whole sweeps");
        const uint64_t tot = ((uint64_t)therm[i] + sweeps[i]) * h->N;
        const long double att = (long double)h->p.walkers * (long double)tot;
        if (att >= 18446744073709551615.0L || h->position + tot < h->position)
            return bfail(b, MUCA_ERR_OVERFLOW, "member " + std::to_string(i) + " would overflow");
    }
    char* hs = static_cast<char*>(b->h_stage);
    std::vector<uint32_t>& form = b->form;
    std::vector<uint64_t>& total = b->total;
    for (uint32_t i = 0; i < count; ++i) {
        b->mode[i] = mode[i];
        b->therm[i] = therm[i];
        b->sweeps[i] = sweeps[i];
        form[i] = kGeneric;
        total[i] = 0;
        if (mode[i] == MUCA_BATCH_SKIP)
            continue;
        muca_instance* h = b->m[i];
        total[i] = (uint64_t)therm[i] + sweeps[i];
        ++active;
        active_blocks += h->wpad / muca::kWave;
        if (const uint32_t cap = h->p.flags & MUCA_FLAG_SWEEPS_PER_LAUNCH_MASK)
            chunk = std::min(chunk, cap);
        compute_thresholds(h->N, h->omega.data(), h->table5.data());
        void* tab = hs + b->off_tables + b->table_off[i];
        const bool wide_ok = !(h->p.flags & MUCA_FLAG_GENERIC_KERNEL) && muca::wide_sweep_supported(h->L) &&
                             fast_table(h->N, h->table5.data(), static_cast<uint32_t*>(tab), 8);
        const bool fast_ok = !wide_ok && !(h->p.flags & MUCA_FLAG_GENERIC_KERNEL) &&
                             (muca::split_sweep_supported(h->L) || muca::fast_sweep_supported(h->L)) &&
                             fast_table(h->N, h->table5.data(), static_cast<uint32_t*>(tab), 5);
        if (wide_ok) {
            form[i] = kWide;
        } else if (fast_ok) {
            form[i] = kFast;  // two-wave or one-wave decided below
        } else {
            device_table(h->N, h->table5.data(), static_cast<uint64_t*>(tab));
            form[i] = kGeneric;
        }
    }
    b->launches = 0;
    if (active == 0) {
        b->pending = true;
        BATCH_HIP(b, hipEventRecord(b->ev_done, b->stream), "hipEventRecord");
        return MUCA_OK;
    }
    // the round's launch plan (muca_host::round_fit / plan_forms): the
    // two-wave form while all of its workgroups fit on the device at once,
    // single or in pairs; otherwise the mixed-longest shape, or with the
    // autotuner the shape it picks
    std::vector<muca_host::RoundMember> rm(count);
    for (uint32_t i = 0; i < count; ++i) {
        if (mode[i] == MUCA_BATCH_SKIP)
            continue;
        const muca_instance* h = b->m[i];
        muca_host::RoundMember& r = rm[i];
        r.active = true;
        r.L = h->L;
        r.blocks = h->wpad / muca::kWave;
        r.walkers = h->p.walkers;
        r.chain = (uint64_t)h->N * total[i];
        r.table = form[i];
        r.forced_fast = (h->p.flags & MUCA_FLAG_FAST_KERNEL) != 0;
        r.split_ok = muca::split_sweep_supported(h->L);
        r.fast_ok = muca::fast_sweep_supported(h->L);
        r.pair_ok = muca::pair_sweep_supported(h->L);
        r.wide_split_ok = muca::wide_split_supported(h->L);
        r.two_wave_bytes = form[i] == kFast && r.split_ok       ? muca::split_lds_bytes(h->L)
                           : form[i] == kWide && r.wide_split_ok ? muca::wide_split_lds_bytes(h->L)
                                                                 : 0u;
        r.fast_waves = r.fast_ok ? muca::fast_waves_per_group(h->L) : 1u;
    }
    const muca_host::RoundFit fit = muca_host::round_fit(rm.data(), count, (uint32_t)b->cus, muca::kLdsPerCu);
    const bool two_wave = fit.two_wave;
    const uint64_t walkers = fit.walkers;
    b->tuning = false;
    b->round_walkers = walkers;
    if (two_wave) {
        b->choice = kTwoWave;
    } else if (b->flags & MUCA_BATCH_AUTOTUNE) {
        if (b->tuned_form >= 0 && 2 * walkers < b->tuned_walkers) {
            b->tuned_form = -1;  // the rounds have thinned out: time the shapes again
            b->tune_step = 0;
        }
        b->tuning = b->tuned_form < 0;
        b->choice = b->tuning ? kTuned[b->tune_step % kNumTuned] : b->tuned_form;
    } else {
        b->choice = kMixedLongest;
    }
    // the kernel form of the choice (the merge-cadence choice keeps the default shape)
    const int shape = b->choice == kTwoMerges ? (two_wave ? kTwoWave : kMixedLongest) : b->choice;
    std::vector<uint32_t> waves(count, 1u);
    muca_host::plan_forms(rm.data(), count, (uint32_t)b->cus, fit, shape, form.data(), waves.data());
    for (uint32_t i = 0; i < count; ++i) {
        const uint32_t L = b->m[i]->L;
        // a launch stays below 2^32 counts per LDS counter of a workgroup
        if (mode[i] != MUCA_BATCH_SKIP)
            chunk = std::min(chunk, muca::max_sweeps_per_launch(L, waves[i]));
    }

    // -- groups and work items; within a group the members with the most
    //    sweeps come first so that their workgroups start first
    std::map<std::pair<uint32_t, uint32_t>, std::vector<uint32_t>> by_group;  // (L, form) -> members
    // (within a round every member of one (L, form) has the same wave count)
    for (uint32_t i = 0; i < count; ++i)
        if (mode[i] != MUCA_BATCH_SKIP)
            by_group[{b->m[i]->L, form[i]}].push_back(i);
    std::vector<Group> groups;
    auto* items = reinterpret_cast<muca::BatchItem*>(hs + b->off_items);
    uint32_t nitems = 0;
    std::string key;
    for (auto it = by_group.rbegin(); it != by_group.rend(); ++it) {  // largest L first
        std::vector<uint32_t>& mem = it->second;
        std::stable_sort(mem.begin(), mem.end(), [&](uint32_t x, uint32_t y) { return total[x] > total[y]; });
        Group G;
        G.L = it->first.first;
        G.form = it->first.second;
        G.waves = waves[mem.front()];
        G.first_item = nitems;
        for (uint32_t i : mem) {
            // a work item is one workgroup: 64 walkers, or for the one-wave
            // form fast_waves_per_group(L) blocks of 64 (for the pair form two)
            // that share one table
            const uint32_t blocks = b->m[i]->wpad / muca::kWave;
            const uint32_t per = (G.form == kFast || G.form == kPair) ? G.waves : 1u;
            for (uint32_t blk = 0; blk < (blocks + per - 1) / per; ++blk)
                items[nitems++] = muca::BatchItem{i, blk};
            key += std::to_string(i) + ":" + std::to_string(total[i]) + ",";
            G.chain = std::max(G.chain, (uint64_t)b->m[i]->N * total[i]);
        }
        G.nitems = nitems - G.first_item;
        key += "|" + std::to_string(G.L) + "/" + std::to_string(G.form) + "/" + std::to_string(G.waves) + ";";
        groups.push_back(G);
    }
    // dispatch order: two-wave groups first, then the others, each kind by its
    // longest chain (muca_order.hip); the starts are staggered where placement
    // can hold a workgroup back -- rounds whose two-wave workgroups do not all
    // fit, and rounds of pair workgroups, each of which needs a whole CU
    b->stagger = !two_wave || fit.use_pairs;
    key += b->stagger ? "s" : "u";
    std::stable_sort(groups.begin(), groups.end(), [](const Group& x, const Group& y) {
        const bool tx = two_wave_form(x.form), ty = two_wave_form(y.form);
        return tx != ty ? tx : x.chain > y.chain;
    });
    if (int rc = ensure_group_streams(b, groups.size()))
        return rc;
    const size_t stage_used = b->stage_bytes;

    // -- device work, chunk by chunk (one chunk unless a member runs more
    //    sweeps than its LDS counters allow per launch)
    uint64_t longest = 0;
    for (uint32_t i = 0; i < count; ++i)
        longest = std::max(longest, total[i]);
    if (b->choice == kTwoMerges && longest > 1)
        chunk = (uint32_t)std::min<uint64_t>(chunk, (longest + 1) / 2);
    b->pending = true;
    auto dev_fail = [&](const char* what, hipError_t e) {
        b->err = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
        return poison_round(b, b->err);
    };
    hipError_t e;
    b->host_in_graph = (b->flags & MUCA_BATCH_GRAPH) && chunk >= longest;
    if (b->host_in_graph) {
        // one captured graph per round shape: clear, upload, sweeps, download,
        // then the host half of the round (merge check, Eq. 4) as a host node
        auto* fargs = reinterpret_cast<muca::FastSweepArgs*>(hs + b->off_fargs);
        auto* gargs = reinterpret_cast<muca::SweepArgs*>(hs + b->off_gargs);
        for (uint32_t i = 0; i < count; ++i) {
            if (mode[i] == MUCA_BATCH_SKIP)
                continue;
            muca_instance* h = b->m[i];
            const uint32_t n = (uint32_t)total[i];
            const char* dtab = static_cast<char*>(b->d_stage) + b->off_tables + b->table_off[i];
            fargs[i] = muca::FastSweepArgs{h->d_spins, h->d_energy, reinterpret_cast<const uint32_t*>(dtab),
                                           b->d_hist + b->hist_off[i], h->position / h->N, h->wpad,
                                           h->p.walkers, h->p.seed, n, therm[i], 0u};
            gargs[i] = muca::SweepArgs{h->d_spins, h->d_energy, reinterpret_cast<const uint64_t*>(dtab),
                                       b->d_hist + b->hist_off[i], h->position / h->N, h->wpad,
                                       h->p.walkers, h->p.seed, n, therm[i], 0u};
        }
        if (b->graph_key != key || !b->exec) {
            drop_graph(b);
            if ((e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return dev_fail("hipStreamBeginCapture", e);
            int rc = MUCA_OK;
            e = muca::launch_fill_u64(b->d_hist, b->hist_words, b->stream);
            if (e == hipSuccess)
                rc = enqueue_round(b, stage_used, groups);
            if (e == hipSuccess && rc == MUCA_OK)
                e = hipMemcpyAsync(b->h_hist, b->d_hist, b->hist_words * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                   b->stream);
            if (e == hipSuccess && rc == MUCA_OK)
                e = hipLaunchHostFunc(b->stream, host_finish_node, b);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
            if (rc != MUCA_OK || e != hipSuccess || e2 != hipSuccess) {
                if (g)
                    (void)hipGraphDestroy(g);
                if (rc != MUCA_OK)
                    return poison_round(b, b->err);
                return dev_fail("batch graph capture", e != hipSuccess ? e : e2);
            }
            b->graph = g;
            if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
                return dev_fail("hipGraphInstantiate", e);
            b->graph_key = key;
        }
        b->launches = (uint32_t)groups.size();
        if ((e = hipEventRecord(b->ev_start, b->stream)) != hipSuccess)
            return dev_fail("hipEventRecord", e);
        if ((e = hipGraphLaunch(b->exec, b->stream)) != hipSuccess)
            return dev_fail("hipGraphLaunch", e);
        if ((e = hipEventRecord(b->ev_stop, b->stream)) != hipSuccess)
            return dev_fail("hipEventRecord", e);
        if ((e = hipEventRecord(b->ev_done, b->stream)) != hipSuccess)
            return dev_fail("hipEventRecord", e);
        return MUCA_OK;
    }
    if ((e = muca::launch_fill_u64(b->d_hist, b->hist_words, b->stream)) != hipSuccess)
        return dev_fail("histogram clear", e);
    if ((e = hipEventRecord(b->ev_start, b->stream)) != hipSuccess)
        return dev_fail("hipEventRecord", e);
    for (uint64_t s0 = 0; s0 < longest; s0 += chunk) {
        auto* fargs = reinterpret_cast<muca::FastSweepArgs*>(hs + b->off_fargs);
        auto* gargs = reinterpret_cast<muca::SweepArgs*>(hs + b->off_gargs);
        std::vector<Group> live;
        for (const Group& G : groups) {
            bool any = false;  // a member of the group still has sweeps in this chunk
            for (uint32_t t = G.first_item; t < G.first_item + G.nitems; ++t)
                any |= total[items[t].member] > s0;
            if (any)
                live.push_back(G);
        }
        for (uint32_t i = 0; i < count; ++i) {
            if (mode[i] == MUCA_BATCH_SKIP)
                continue;
            muca_instance* h = b->m[i];
            const uint64_t left = total[i] > s0 ? total[i] - s0 : 0;
            const uint32_t n = (uint32_t)std::min<uint64_t>(left, chunk);
            const uint32_t th = s0 >= therm[i] ? 0u : (uint32_t)std::min<uint64_t>(therm[i] - s0, n);
            const char* dtab = static_cast<char*>(b->d_stage) + b->off_tables + b->table_off[i];
            fargs[i] = muca::FastSweepArgs{h->d_spins, h->d_energy, reinterpret_cast<const uint32_t*>(dtab),
                                           b->d_hist + b->hist_off[i], h->position / h->N + s0, h->wpad,
                                           h->p.walkers, h->p.seed, n, th, 0u};
            gargs[i] = muca::SweepArgs{h->d_spins, h->d_energy, reinterpret_cast<const uint64_t*>(dtab),
                                       b->d_hist + b->hist_off[i], h->position / h->N + s0, h->wpad,
                                       h->p.walkers, h->p.seed, n, th, 0u};
        }
        if (enqueue_round(b, stage_used, live) != MUCA_OK)
            return poison_round(b, b->err);
        b->launches += (uint32_t)live.size();
        // a further chunk rewrites the staged arguments once the upload is done
        if (s0 + chunk < longest && (e = hipStreamSynchronize(b->stream)) != hipSuccess)
            return dev_fail("batch stream", e);
    }
    if ((e = hipEventRecord(b->ev_stop, b->stream)) != hipSuccess)
        return dev_fail("hipEventRecord", e);
    if ((e = hipMemcpyAsync(b->h_hist, b->d_hist, b->hist_words * sizeof(uint64_t), hipMemcpyDeviceToHost,
                            b->stream)) != hipSuccess)
        return dev_fail("batch histogram download", e);
    if ((e = hipEventRecord(b->ev_done, b->stream)) != hipSuccess)
        return dev_fail("hipEventRecord", e);
    return MUCA_OK;
}

// No C++ exception leaves the C ABI: a failed host allocation while a round
// is set up is reported, and a round it interrupted poisons its members.
int muca_batch_submit(muca_batch* b, const uint32_t* mode, const uint32_t* therm,
                      const uint32_t* sweeps)
{
    int code = MUCA_ERR_STATE;
    try {
        return muca_batch_submit_impl(b, mode, therm, sweeps);
    } catch (const std::bad_alloc&) {
        code = MUCA_ERR_OUT_OF_MEMORY;
    } catch (...) {
    }
    // a round that had started: let its device work end, then poison its members
    if (b->pending) {
        (void)hipStreamSynchronize(b->stream);
        poison_round(b, "host exception while the round was set up");
    }
    return bfail(b, code, code == MUCA_ERR_OUT_OF_MEMORY ? "host allocation failed" : "unexpected host exception");
}

int muca_batch_query(muca_batch* b)
{
    if (!b)
        return MUCA_ERR_INVALID_ARG;
    if (!b->pending)
        return bfail(b, MUCA_ERR_STATE, "no submitted round");
    const hipError_t e = hipEventQuery(b->ev_done);
    if (e == hipErrorNotReady)
        return MUCA_PENDING;
    if (e != hipSuccess) {
        b->err = std::string("hipEventQuery: ") + hipGetErrorName(e);
        return poison_round(b, b->err);
    }
    return MUCA_OK;
}

int muca_batch_finish(muca_batch* b, muca_info* infos)
{
    if (!b)
        return MUCA_ERR_INVALID_ARG;
    if (!b->pending)
        return bfail(b, MUCA_ERR_STATE, "no submitted round");
    hipError_t e = hipEventSynchronize(b->ev_done);
    if (e != hipSuccess) {
        b->err = std::string("hipEventSynchronize: ") + hipGetErrorName(e);
        return poison_round(b, b->err);
    }
    b->pending = false;
    const uint32_t count = (uint32_t)b->m.size();
    float ms = 0.0f;
    if (b->launches) {
        if ((e = hipEventElapsedTime(&ms, b->ev_start, b->ev_stop)) != hipSuccess)
            return bfail(b, MUCA_ERR_DEVICE, std::string("hipEventElapsedTime: ") + hipGetErrorName(e));
    }

    // -- host: per-member results (already applied by the graph's host node,
    //    whose device time the round's kernel_ms then includes)
    int result = MUCA_OK;
    if (b->host_in_graph) {
        result = b->host_rc;
        if (result != MUCA_OK)
            b->err = b->host_err;
        for (uint32_t i = 0; i < count; ++i)
            if (b->mode[i] != MUCA_BATCH_SKIP) {
                b->round_infos[i].kernel_ms = ms;
                b->m[i]->last.kernel_ms = ms;
            }
    } else {
        std::string why;
        result = finish_members(b, ms, b->round_infos, &why);
        if (result != MUCA_OK)
            b->err = why;
    }
    uint64_t attempts = 0;
    for (uint32_t i = 0; i < count; ++i) {
        if (b->mode[i] == MUCA_BATCH_SKIP)
            continue;
        if (infos)
            infos[i] = b->round_infos[i];
        attempts += (uint64_t)b->m[i]->p.walkers * b->m[i]->N * b->total[i];
    }
    if (b->launches && b->tuning && ms > 0.0f) {
        b->tuned_rate[b->choice] = (double)attempts / ms;
        if (++b->tune_step >= kNumTuned) {
            int best = kTuned[0];
            for (int c : kTuned)
                if (b->tuned_rate[c] > b->tuned_rate[best])
                    best = c;
            b->tuned_form = best;
            b->tuned_walkers = b->round_walkers;
        }
    }
    if (b->launches)
        ++b->round;
    return result;
}

int muca_batch_run(muca_batch* b, const uint32_t* mode, const uint32_t* therm,
                   const uint32_t* sweeps, muca_info* infos)
{
    if (int rc = muca_batch_submit(b, mode, therm, sweeps))
        return rc;
    return muca_batch_finish(b, infos);
}

}  // extern "C"
