// muca_server.cpp -- continuous batching of multicanonical solves
// (include/muca.h, muca_server_*).
//
// A request is one complete solve of Sec. 2.2: weight iterations (Eq. 4) until
// the histogram is flat enough, then a production run at the frozen weights,
// whose histogram gives ln g (Sec. 3.3).  The server keeps every admitted
// request resident on the device -- lattices, energies, histogram, weights --
// until it is done, and runs the admitted requests together:
//
//   queue    requests wait in arrival order (or, with the smallest-first
//            policy, the one of least estimated work goes next, unless one
//            has waited longer than the configured bound); the next one
//            is admitted when its device state (muca_state_bytes) fits in the
//            free part of the server's arena and the walker budget allows it;
//   lanes    admitted requests are grouped by L; each lane is one batch
//            (muca_batch) on its own stream, so lanes of different L run at
//            the same time and each lane starts its next round as soon as its
//            last one ends, independently of the others;
//   rounds   in a lane round every member runs one step of its own schedule:
//            a weight iteration, or a production slice of at most iter_sweeps
//            sweeps (production histograms are summed on the host), so the
//            members of a lane take equally long per round;
//   retire   a finished request gets ln g from the summed production
//            histogram, leaves its lane and gives its arena space back.
//
// Each request's chain depends only on its own (L, walkers, seed, weights,
// sweep counter), so its results are bit-identical to running it alone with
// muca_iterate / muca_production / muca_log_dos.
//
// Device memory of requests comes from one arena allocated when the server is
// created; nothing is allocated or freed on the device while the server runs
// (beyond a lane's staging growing), so no call waits for other lanes' work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "muca.h"
#include "muca_internal.h"

namespace {

thread_local std::string g_server_error;

using muca_host::Arena;

enum Phase : uint32_t { kQueued = 0, kIterating = 1, kProducing = 2, kDone = 3 };

struct Request {
    uint64_t ticket = 0;
    muca_request q{};
    Phase phase = kQueued;
    muca_instance* h = nullptr;
    size_t bytes = 0, arena_off = 0;
    uint32_t iterations = 0;
    double flatness = 0.0;
    uint32_t prod_therm_left = 0, prod_left = 0;
    std::vector<uint64_t> acc;  // summed production histogram
    std::vector<double> ln_g;
    int status = MUCA_OK;
    std::string err;
    uint64_t attempts = 0;
    double t_submit = 0, t_admit = -1, t_weights = -1, t_done = -1;
    double work = 0;  // estimated attempts (muca_host::solve_work_estimate)
};

struct Lane {
    uint32_t L = 0;
    hipStream_t stream = nullptr;
    muca_batch* batch = nullptr;
    std::vector<Request*> members;  // the batch's members, in its order
    std::vector<Request*> joining;  // admitted while a round ran; join the next one
    bool dirty = true;  // membership changed since the batch last saw it
    bool in_flight = false;
    std::vector<uint32_t> mode, therm, sweeps;
};

}  // namespace

struct muca_server {
    muca_server_config cfg{};
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    char* arena_base = nullptr;
    Arena arena;
    uint64_t next_ticket = 1;
    std::deque<Request*> queue;
    std::map<uint64_t, std::unique_ptr<Request>> requests;  // until taken
    std::map<uint32_t, Lane> lanes;                         // by L
    std::vector<muca_instance*> graveyard;  // retired, destroyed when no lane runs
    uint64_t active_walkers = 0;
    uint64_t attempts = 0;
    uint64_t completed = 0, admitted = 0;
    std::string err;
};

namespace {

int sfail(muca_server* s, int code, const std::string& msg)
{
    if (s)
        s->err = msg;
    else
        g_server_error = msg;
    return code;
}

double now_s(const muca_server* s)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

bool request_valid(const muca_request* q, std::string* why)
{
    muca_params p{q->L, q->walkers, q->seed, q->flags};
    if (muca_state_bytes(&p) == 0) {
        *why = "invalid instance parameters (L even in [4, 128], walkers >= 1)";
        return false;
    }
    if (q->iter_sweeps == 0) {
        *why = "iter_sweeps must be >= 1";
        return false;
    }
    if (!(q->min_flatness >= 0.0 && q->min_flatness <= 1.0)) {
        *why = "min_flatness must lie in [0, 1]";
        return false;
    }
    return true;
}

void destroy_graveyard(muca_server* s)
{
    for (muca_instance* h : s->graveyard)
        muca_destroy(h);
    s->graveyard.clear();
}

// Ends a request: ln g from the summed production histogram, instance retired.
void retire(muca_server* s, Request* r, int status, const std::string& why)
{
    muca_instance* h = r->h;
    if (status == MUCA_OK && h) {
        std::copy(r->acc.begin(), r->acc.end(), h->hist.begin());
        r->ln_g.assign((size_t)h->N + 1, 0.0);
        status = muca_log_dos(h, 0, r->ln_g.data(), r->ln_g.size());
        if (status != MUCA_OK) {
            r->err = muca_last_error(h);
            r->ln_g.clear();
        }
    } else {
        r->err = why;
    }
    r->status = status;
    r->phase = kDone;
    r->t_done = now_s(s);
    if (h) {
        s->graveyard.push_back(h);
        r->h = nullptr;
        s->arena.release(r->arena_off, r->bytes);
        s->active_walkers -= r->q.walkers;
    }
    r->acc.clear();
    r->acc.shrink_to_fit();
    ++s->completed;
}

// Admits queued requests while the next one fits: in arrival order, or with
// MUCA_SERVE_SMALLEST_FIRST the one of least estimated work first (ties in
// arrival order) unless a request has waited longer than max_wait_s
// (muca_host::admission_pick).  The picked request is moved to the front and
// blocks the queue until it fits.
int admit(muca_server* s)
{
    std::vector<muca_host::QueuedJob> jobs;
    while (!s->queue.empty()) {
        if (s->cfg.policy == MUCA_SERVE_SMALLEST_FIRST) {
            jobs.clear();
            for (const Request* r : s->queue)
                jobs.push_back({r->work, r->t_submit});
            const double wait = s->cfg.max_wait_s > 0.0 ? s->cfg.max_wait_s : 30.0;
            const size_t i = muca_host::admission_pick(jobs.data(), jobs.size(), true, now_s(s), wait);
            if (i != 0) {
                Request* b = s->queue[i];
                s->queue.erase(s->queue.begin() + (std::ptrdiff_t)i);
                s->queue.push_front(b);
            }
        }
        Request* r = s->queue.front();
        if (s->cfg.max_active_walkers && s->active_walkers > 0 &&
            s->active_walkers + r->q.walkers > s->cfg.max_active_walkers)
            return MUCA_OK;
        muca_params p{r->q.L, r->q.walkers, r->q.seed, r->q.flags};
        r->bytes = muca_state_bytes(&p);
        size_t off = 0;
        if (!s->arena.alloc(r->bytes, &off)) {
            if (s->arena.used() == 0) {  // can never fit
                s->queue.pop_front();
                retire(s, r, MUCA_ERR_OUT_OF_MEMORY, "request larger than the server's memory cap");
                continue;
            }
            return MUCA_OK;
        }
        s->queue.pop_front();
        r->arena_off = off;
        muca_instance* h = nullptr;
        const int rc = muca_create(&p, nullptr, s->arena_base + off, r->bytes, &h);
        if (rc != MUCA_OK) {
            s->arena.release(off, r->bytes);
            retire(s, r, rc, std::string("muca_create: ") + muca_last_error(nullptr));
            continue;
        }
        r->h = h;
        r->phase = kIterating;
        r->t_admit = now_s(s);
        r->prod_therm_left = r->q.prod_therm;
        r->prod_left = r->q.prod_sweeps;
        r->acc.assign((size_t)h->N + 1, 0);
        s->active_walkers += r->q.walkers;
        ++s->admitted;
        Lane& lane = s->lanes[r->q.L];
        lane.L = r->q.L;
        lane.joining.push_back(r);
    }
    return MUCA_OK;
}

// Host half of a finished lane round: advance every member's schedule.
void lane_collect(muca_server* s, Lane& lane, const std::vector<muca_info>& infos, int rc)
{
    // lane.members are exactly the members of the round that ended (joiners
    // wait in lane.joining), so infos, mode, therm and sweeps line up with them
    std::vector<Request*> keep;
    if (lane.mode.size() != lane.members.size() || infos.size() != lane.members.size())
        rc = MUCA_ERR_STATE;  // cannot happen: the round's arrays are sized at launch
    for (size_t i = 0; i < lane.members.size(); ++i) {
        Request* r = lane.members[i];
        if (rc != MUCA_OK || r->h->poisoned) {
            retire(s, r, rc == MUCA_ERR_STATE ? rc : MUCA_ERR_DEVICE, std::string("round failed: ") + r->h->err);
            continue;
        }
        const muca_info& in = infos[i];
        r->attempts += in.attempts;
        s->attempts += in.attempts;
        if (lane.mode[i] == MUCA_BATCH_ITERATE) {
            ++r->iterations;
            r->flatness = in.flatness;
            const bool flat = in.flatness >= r->q.min_flatness;
            if (flat || (r->q.max_iterations && r->iterations >= r->q.max_iterations)) {
                r->t_weights = now_s(s);
                r->phase = kProducing;
                if (!flat)
                    r->status = MUCA_ERR_NOT_CONVERGED;  // kept unless a later error replaces it
            }
        } else {
            const uint32_t th = lane.therm[i], sw = lane.sweeps[i];
            r->prod_therm_left -= th;
            r->prod_left -= sw;
            const uint64_t* H = r->h->hist.data();
            for (size_t k = 0; k < r->acc.size(); ++k)
                r->acc[k] += H[k];
        }
        if (r->phase == kProducing && r->prod_therm_left == 0 && r->prod_left == 0) {
            const int st = r->status;
            retire(s, r, MUCA_OK, "");
            if (st != MUCA_OK && r->status == MUCA_OK)
                r->status = st;
            continue;
        }
        keep.push_back(r);
    }
    if (keep.size() != lane.members.size())
        lane.dirty = true;
    lane.members.swap(keep);
}

int lane_launch(muca_server* s, Lane& lane)
{
    if (!lane.joining.empty()) {
        lane.members.insert(lane.members.end(), lane.joining.begin(), lane.joining.end());
        lane.joining.clear();
        lane.dirty = true;
    }
    const size_t n = lane.members.size();
    if (n == 0)
        return MUCA_OK;
    std::vector<muca_instance*> hs(n);
    for (size_t i = 0; i < n; ++i)
        hs[i] = lane.members[i]->h;
    if (!lane.stream && hipStreamCreateWithFlags(&lane.stream, hipStreamNonBlocking) != hipSuccess)
        return sfail(s, MUCA_ERR_DEVICE, "hipStreamCreate failed");
    if (!lane.batch) {
        if (int rc = muca_batch_create(hs.data(), (uint32_t)n, lane.stream, s->cfg.batch_flags, &lane.batch))
            return sfail(s, rc, std::string("muca_batch_create: ") + muca_batch_last_error(nullptr));
    } else if (lane.dirty) {
        if (int rc = muca_batch_set_members(lane.batch, hs.data(), (uint32_t)n))
            return sfail(s, rc, std::string("muca_batch_set_members: ") + muca_batch_last_error(lane.batch));
    }
    lane.dirty = false;
    lane.mode.assign(n, MUCA_BATCH_SKIP);
    lane.therm.assign(n, 0);
    lane.sweeps.assign(n, 0);
    for (size_t i = 0; i < n; ++i) {
        const Request* r = lane.members[i];
        const uint32_t slice = r->q.iter_sweeps;
        if (r->phase == kIterating) {
            lane.mode[i] = MUCA_BATCH_ITERATE;
            lane.therm[i] = r->q.iter_therm;
            lane.sweeps[i] = r->q.iter_sweeps;
        } else {
            lane.mode[i] = MUCA_BATCH_PRODUCTION;
            const uint32_t th = std::min(r->prod_therm_left, slice);
            lane.therm[i] = th;
            lane.sweeps[i] = std::min(r->prod_left, slice - th);
        }
    }
    if (int rc = muca_batch_submit(lane.batch, lane.mode.data(), lane.therm.data(), lane.sweeps.data()))
        return sfail(s, rc, std::string("muca_batch_submit: ") + muca_batch_last_error(lane.batch));
    lane.in_flight = true;
    return MUCA_OK;
}

void release(muca_server* s)
{
    if (!s)
        return;
    for (auto& kv : s->lanes) {
        Lane& lane = kv.second;
        if (lane.in_flight && lane.batch)
            (void)muca_batch_finish(lane.batch, nullptr);
        if (lane.batch)
            muca_batch_destroy(lane.batch);
        if (lane.stream)
            (void)hipStreamDestroy(lane.stream);
    }
    for (auto& kv : s->requests)
        if (kv.second->h)
            s->graveyard.push_back(kv.second->h);
    destroy_graveyard(s);
    if (s->arena_base)
        (void)hipFree(s->arena_base);
    delete s;
}

}  // namespace

extern "C" {

int muca_server_create(const muca_server_config* cfg, muca_server** out)
{
    if (!out)
        return sfail(nullptr, MUCA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg || cfg->mem_cap_bytes == 0)
        return sfail(nullptr, MUCA_ERR_INVALID_ARG, "a memory cap is required");
    if (cfg->batch_flags & ~(uint32_t)(MUCA_BATCH_GRAPH | MUCA_BATCH_AUTOTUNE))
        return sfail(nullptr, MUCA_ERR_INVALID_ARG, "unknown batch flag");
    if (cfg->policy > MUCA_SERVE_SMALLEST_FIRST)
        return sfail(nullptr, MUCA_ERR_INVALID_ARG, "unknown admission policy");
    if (!(cfg->max_wait_s >= 0.0))
        return sfail(nullptr, MUCA_ERR_INVALID_ARG, "max_wait_s must be >= 0");
    muca_server* s = new (std::nothrow) muca_server();
    if (!s)
        return sfail(nullptr, MUCA_ERR_OUT_OF_MEMORY, "host allocation failed");
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return sfail(nullptr, MUCA_ERR_DEVICE, "hipGetDevice failed");
    }
    if (hipMalloc((void**)&s->arena_base, cfg->mem_cap_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return sfail(nullptr, MUCA_ERR_OUT_OF_MEMORY, "arena allocation failed");
    }
    s->arena.reset(cfg->mem_cap_bytes);
    *out = s;
    return MUCA_OK;
}

static int muca_server_submit_impl(muca_server* s, const muca_request* q, uint64_t* ticket)
{
    if (!s || !q || !ticket)
        return MUCA_ERR_INVALID_ARG;
    std::string why;
    if (!request_valid(q, &why))
        return sfail(s, MUCA_ERR_INVALID_ARG, why);
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r)
        return sfail(s, MUCA_ERR_OUT_OF_MEMORY, "host allocation failed");
    r->ticket = s->next_ticket++;
    r->q = *q;
    r->t_submit = now_s(s);
    r->work = muca_host::solve_work_estimate(q->L, q->walkers, q->iter_therm, q->iter_sweeps, q->max_iterations,
                                             q->prod_therm, q->prod_sweeps);
    Request* raw = r.get();
    s->requests[raw->ticket] = std::move(r);
    try {
        s->queue.push_back(raw);
    } catch (...) {
        s->requests.erase(raw->ticket);  // the queue never saw it
        throw;
    }
    *ticket = raw->ticket;
    return MUCA_OK;
}

// No C++ exception leaves the C ABI: a failed host allocation is reported.
int muca_server_submit(muca_server* s, const muca_request* q, uint64_t* ticket)
{
    try {
        return muca_server_submit_impl(s, q, ticket);
    } catch (const std::bad_alloc&) {
        return sfail(s, MUCA_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return sfail(s, MUCA_ERR_STATE, "unexpected host exception");
    }
}

static int muca_server_progress_impl(muca_server* s, uint32_t* events)
{
    if (!s)
        return MUCA_ERR_INVALID_ARG;
    if (hipSetDevice(s->device) != hipSuccess)
        return sfail(s, MUCA_ERR_DEVICE, "hipSetDevice failed");
    uint32_t ev = 0;
    bool any_running = false;
    // finished rounds first: they free slots and memory
    for (auto& kv : s->lanes) {
        Lane& lane = kv.second;
        if (!lane.in_flight)
            continue;
        int rc = muca_batch_query(lane.batch);
        if (rc == MUCA_PENDING) {
            any_running = true;
            continue;
        }
        std::vector<muca_info> infos(lane.members.size());
        if (rc == MUCA_OK)
            rc = muca_batch_finish(lane.batch, infos.data());
        lane.in_flight = false;
        lane_collect(s, lane, infos, rc);
        ++ev;
    }
    if (!any_running && !s->graveyard.empty())
        destroy_graveyard(s);
    admit(s);
    for (auto& kv : s->lanes) {
        Lane& lane = kv.second;
        if (lane.in_flight || (lane.members.empty() && lane.joining.empty()))
            continue;
        if (int rc = lane_launch(s, lane)) {
            for (Request* r : lane.members)
                retire(s, r, rc, s->err);
            for (Request* r : lane.joining)
                retire(s, r, rc, s->err);
            lane.members.clear();
            lane.joining.clear();
            lane.dirty = true;
            return rc;
        }
        ++ev;
    }
    if (events)
        *events = ev;
    return MUCA_OK;
}

// No C++ exception leaves the C ABI: a failed host allocation is reported.
int muca_server_progress(muca_server* s, uint32_t* events)
{
    try {
        return muca_server_progress_impl(s, events);
    } catch (const std::bad_alloc&) {
        return sfail(s, MUCA_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return sfail(s, MUCA_ERR_STATE, "unexpected host exception");
    }
}

int muca_server_take(muca_server* s, uint64_t ticket, muca_result* res, double* ln_g, size_t n)
{
    if (!s || !res)
        return MUCA_ERR_INVALID_ARG;
    auto it = s->requests.find(ticket);
    if (it == s->requests.end())
        return sfail(s, MUCA_ERR_INVALID_ARG, "unknown ticket");
    Request* r = it->second.get();
    if (r->phase != kDone)
        return MUCA_PENDING;
    const size_t N1 = (size_t)r->q.L * r->q.L + 1;
    if (ln_g && n != N1)
        return sfail(s, MUCA_ERR_INVALID_ARG, "ln_g must hold L*L+1 values");
    muca_result o{};
    o.ticket = r->ticket;
    o.status = r->status;
    o.iterations = r->iterations;
    o.flatness = r->flatness;
    o.attempts = r->attempts;
    o.t_submit = r->t_submit;
    o.t_admit = r->t_admit;
    o.t_weights = r->t_weights;
    o.t_done = r->t_done;
    *res = o;
    if (ln_g) {
        if (r->ln_g.size() == N1)
            std::memcpy(ln_g, r->ln_g.data(), N1 * sizeof(double));
        else
            std::fill(ln_g, ln_g + N1, 0.0);
    }
    s->requests.erase(it);
    return MUCA_OK;
}

int muca_server_stats(const muca_server* s, muca_server_counters* out)
{
    if (!s || !out)
        return MUCA_ERR_INVALID_ARG;
    muca_server_counters o{};
    o.queued = (uint32_t)s->queue.size();
    for (const auto& kv : s->lanes)
        o.active += (uint32_t)(kv.second.members.size() + kv.second.joining.size());
    o.completed = s->completed;
    o.admitted = s->admitted;
    o.resident_bytes = s->arena.used();
    o.active_walkers = s->active_walkers;
    o.attempts = s->attempts;
    o.clock_s = now_s(s);
    *out = o;
    return MUCA_OK;
}

int muca_server_destroy(muca_server* s)
{
    release(s);
    return MUCA_OK;
}

const char* muca_server_last_error(const muca_server* s)
{
    return s ? s->err.c_str() : g_server_error.c_str();
}

}  // extern "C"
