// CPU stand-in for the HIP runtime and for libmuca's kernels (see
// hip/hip_runtime.h).  Test infrastructure: the host half of libmuca is linked
// against this file and driven under the sanitizers.
//
// Runtime model
//   * allocations are host memory (from 1 GiB on, mapped pages that cost
//     nothing until touched), registered with their size and kind (device or
//     pinned host), so that every copy and every stand-in kernel checks that
//     what it touches lies inside one live allocation of the right kind;
//   * a stream is a worker thread that runs its work in order; an event
//     records a point in a stream; a stream that waits for an event waits for
//     that point;
//   * capture records a stream's work (and that of the streams that join it
//     through events) into a graph; a graph launch runs the recorded work, in
//     recorded order, on the launching stream; host functions run on the
//     stream's worker and hold back later work until they return;
//   * hipFree and hipHostFree wait for all streams, as HIP's do, and count
//     the times they had work to wait for (with CPU_HIP_FREE_NOWAIT=1 they
//     free at once instead, so that work still queued on freed memory shows).
//
// Kernel model
//   Each stand-in kernel checks its arguments the way the real kernel uses
//   them (lattice, energies, table, histogram, work items), touches every
//   word it would touch, and adds N counts per recorded sweep of every live
//   walker to the histogram, spread evenly over the first K reachable bins,
//   K = min(N + 1, 16 * 2^(sweep / 200)) for each sweep: the histogram sum is the one the
//   host checks, and an instance needs about log2(N / 16) weight iterations
//   before its histogram is flat.  Kernel time is simulated: the worker sleeps
//   for attempts / CPU_HIP_RATE seconds (default 4e12 attempts/s).
#include "hip/hip_runtime.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include <sys/mman.h>

#include "muca_device.h"

namespace {

[[noreturn]] void die(const char* what, const void* p = nullptr, size_t n = 0)
{
    std::fprintf(stderr, "cpu_hip: %s (%p, %zu bytes)\n", what, p, n);
    std::fflush(stderr);
    std::abort();
}

// -- allocations -----------------------------------------------------------

enum Kind { kDevice = 1, kPinned = 2 };

struct Alloc {
    size_t bytes;
    Kind kind;
    bool mapped;  // a large allocation, mapped on demand (the server's arena)
};

constexpr size_t kMapFrom = size_t(1) << 30;

std::mutex g_alloc_m;
std::map<uintptr_t, Alloc> g_allocs;
std::atomic<uint64_t> g_free_waits{0};

void check_range(const void* p, size_t bytes, Kind kind, const char* what)
{
    if (bytes == 0)
        return;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    std::lock_guard<std::mutex> lk(g_alloc_m);
    auto it = g_allocs.upper_bound(a);
    if (it == g_allocs.begin())
        die(what, p, bytes);
    --it;
    if (a + bytes > it->first + it->second.bytes || it->second.kind != kind)
        die(what, p, bytes);
}

bool is_kind(const void* p, Kind kind)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    std::lock_guard<std::mutex> lk(g_alloc_m);
    auto it = g_allocs.upper_bound(a);
    if (it == g_allocs.begin())
        return false;
    --it;
    return a < it->first + it->second.bytes && it->second.kind == kind;
}

hipError_t do_alloc(void** p, size_t bytes, Kind kind)
{
    if (!p)
        return hipErrorInvalidValue;
    void* q = nullptr;
    const bool mapped = bytes >= kMapFrom;
    if (mapped) {
        q = mmap(nullptr, bytes, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
        if (q == MAP_FAILED)
            return hipErrorOutOfMemory;
    } else if (posix_memalign(&q, 256, bytes ? bytes : 1) != 0) {
        return hipErrorOutOfMemory;
    }
    {
        std::lock_guard<std::mutex> lk(g_alloc_m);
        g_allocs[reinterpret_cast<uintptr_t>(q)] = Alloc{bytes ? bytes : 1, kind, mapped};
    }
    *p = q;
    return hipSuccess;
}

void wait_all_streams();

hipError_t do_free(void* p, Kind kind)
{
    if (!p)
        return hipSuccess;
    // CPU_HIP_FREE_NOWAIT=1: free at once, so that queued work that still
    // uses the memory trips the sanitizer or the range checks
    static const bool nowait = [] {
        const char* v = std::getenv("CPU_HIP_FREE_NOWAIT");
        return v && v[0] == '1';
    }();
    if (!nowait)
        wait_all_streams();
    Alloc a{};
    {
        std::lock_guard<std::mutex> lk(g_alloc_m);
        auto it = g_allocs.find(reinterpret_cast<uintptr_t>(p));
        if (it == g_allocs.end() || it->second.kind != kind)
            die("free of a pointer that is not a live allocation of this kind", p);
        a = it->second;
        g_allocs.erase(it);
    }
    if (a.mapped)
        munmap(p, a.bytes);
    else
        std::free(p);
    return hipSuccess;
}

}  // namespace

// -- streams, events, graphs ----------------------------------------------

struct ihipGraph {
    std::vector<std::function<void()>> ops;
    bool open = true;
    uint64_t id = 0;
    ihipStream_t* origin = nullptr;
    // joined streams: last op recorded on each, and how far the origin has
    // waited for it
    std::map<ihipStream_t*, std::pair<uint64_t, uint64_t>> joined;
};

struct hipGraphExec {
    std::vector<std::function<void()>> ops;
    std::atomic<int> queued{0};
};

struct ihipEvent_t {
    std::mutex m;
    std::condition_variable cv;
    uint64_t recorded = 0, done = 0;
    std::chrono::steady_clock::time_point t{};
    bool timing = true;
    // a record made during a capture: the capture's id, its stream, the op count there
    uint64_t capture_id = 0;
    ihipStream_t* capture_stream = nullptr;
    uint64_t capture_seq = 0;
};

struct ihipStream_t {
    std::mutex m;
    std::condition_variable cv;
    std::deque<std::function<void()>> q;
    uint64_t enq = 0, fin = 0;
    bool stop = false;
    std::thread th;
    ihipGraph* capture = nullptr;
    uint64_t capture_seq = 0;  // ops recorded on this stream in the open capture

    ihipStream_t()
    {
        th = std::thread([this] { run(); });
    }
    void run()
    {
        for (;;) {
            std::function<void()> f;
            {
                std::unique_lock<std::mutex> lk(m);
                cv.wait(lk, [this] { return stop || !q.empty(); });
                if (q.empty())
                    return;
                f = std::move(q.front());
                q.pop_front();
            }
            f();
            {
                std::lock_guard<std::mutex> lk(m);
                ++fin;
            }
            cv.notify_all();
        }
    }
    void push(std::function<void()> f)
    {
        {
            std::lock_guard<std::mutex> lk(m);
            q.push_back(std::move(f));
            ++enq;
        }
        cv.notify_all();
    }
    void drain()
    {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [this] { return fin == enq; });
    }
    bool idle()
    {
        std::lock_guard<std::mutex> lk(m);
        return fin == enq;
    }
};

namespace {

std::mutex g_streams_m;
std::vector<ihipStream_t*> g_streams;
ihipStream_t* g_null_stream = nullptr;
std::mutex g_capture_m;
std::map<uint64_t, ihipGraph*> g_open_captures;
uint64_t g_next_capture = 1;
thread_local hipError_t g_last_error = hipSuccess;

ihipStream_t* resolve(hipStream_t s)
{
    if (s)
        return s;
    std::lock_guard<std::mutex> lk(g_streams_m);
    if (!g_null_stream) {
        g_null_stream = new ihipStream_t();
        g_streams.push_back(g_null_stream);
    }
    return g_null_stream;
}

void wait_all_streams()
{
    std::vector<ihipStream_t*> all;
    {
        std::lock_guard<std::mutex> lk(g_streams_m);
        all = g_streams;
    }
    bool waited = false;
    for (ihipStream_t* s : all) {
        if (!s->idle())
            waited = true;
        s->drain();
    }
    if (waited)
        ++g_free_waits;
}

// Work on stream s: recorded into its capture, or queued.
void submit(ihipStream_t* s, std::function<void()> f)
{
    if (s->capture) {
        s->capture->ops.push_back(std::move(f));
        ++s->capture_seq;
        if (s != s->capture->origin)
            s->capture->joined[s].first = s->capture_seq;
        return;
    }
    s->push(std::move(f));
}

double rate()
{
    static const double r = [] {
        const char* v = std::getenv("CPU_HIP_RATE");
        return v ? std::atof(v) : 4e12;
    }();
    return r;
}

void simulate(double attempts)
{
    if (rate() > 0.0 && attempts > 0.0)
        std::this_thread::sleep_for(std::chrono::duration<double>(attempts / rate()));
}

}  // namespace

extern "C++" {

hipError_t hipGetDevice(int* device)
{
    if (!device)
        return hipErrorInvalidValue;
    *device = 0;
    return hipSuccess;
}

hipError_t hipSetDevice(int device) { return device == 0 ? hipSuccess : hipErrorInvalidValue; }

hipError_t hipDeviceGetAttribute(int* value, hipDeviceAttribute_t attr, int device)
{
    if (!value || device != 0 || attr != hipDeviceAttributeMultiprocessorCount)
        return hipErrorInvalidValue;
    const char* c = std::getenv("CPU_HIP_CUS");
    *value = c ? std::atoi(c) : 256;
    return hipSuccess;
}

hipError_t hipGetLastError(void)
{
    const hipError_t e = g_last_error;
    g_last_error = hipSuccess;
    return e;
}

const char* hipGetErrorName(hipError_t e)
{
    switch (e) {
    case hipSuccess:
        return "hipSuccess";
    case hipErrorInvalidValue:
        return "hipErrorInvalidValue";
    case hipErrorOutOfMemory:
        return "hipErrorOutOfMemory";
    case hipErrorNotReady:
        return "hipErrorNotReady";
    default:
        return "hipErrorUnknown";
    }
}

const char* hipGetErrorString(hipError_t e) { return hipGetErrorName(e); }

hipError_t hipMalloc(void** p, size_t bytes) { return do_alloc(p, bytes, kDevice); }
hipError_t hipFree(void* p) { return do_free(p, kDevice); }
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) { return do_alloc(p, bytes, kPinned); }
hipError_t hipHostFree(void* p) { return do_free(p, kPinned); }

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s)
{
    if (kind == hipMemcpyHostToDevice) {
        check_range(dst, bytes, kDevice, "host-to-device copy: destination is not device memory");
        if (is_kind(src, kDevice))
            die("host-to-device copy from device memory", src, bytes);
    } else if (kind == hipMemcpyDeviceToHost) {
        check_range(src, bytes, kDevice, "device-to-host copy: source is not device memory");
        if (is_kind(dst, kDevice))
            die("device-to-host copy into device memory", dst, bytes);
    } else if (kind == hipMemcpyDeviceToDevice) {
        check_range(src, bytes, kDevice, "device copy: source");
        check_range(dst, bytes, kDevice, "device copy: destination");
    }
    submit(resolve(s), [dst, src, bytes, kind] {
        // checked again when it runs: the memory may have been freed meanwhile
        if (kind == hipMemcpyHostToDevice)
            check_range(dst, bytes, kDevice, "host-to-device copy ran after its destination was freed");
        if (kind == hipMemcpyDeviceToHost)
            check_range(src, bytes, kDevice, "device-to-host copy ran after its source was freed");
        std::memcpy(dst, src, bytes);
    });
    return hipSuccess;
}

hipError_t hipStreamCreate(hipStream_t* s) { return hipStreamCreateWithFlags(s, 0); }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int)
{
    if (!s)
        return hipErrorInvalidValue;
    ihipStream_t* t = new ihipStream_t();
    std::lock_guard<std::mutex> lk(g_streams_m);
    g_streams.push_back(t);
    *s = t;
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s)
{
    if (!s)
        return hipErrorInvalidValue;
    if (s->capture)
        die("stream destroyed during a capture");
    s->drain();
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
    }
    s->cv.notify_all();
    s->th.join();
    {
        std::lock_guard<std::mutex> lk(g_streams_m);
        g_streams.erase(std::remove(g_streams.begin(), g_streams.end(), s), g_streams.end());
    }
    delete s;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s)
{
    ihipStream_t* t = resolve(s);
    if (t->capture)
        return hipErrorStreamCaptureUnsupported;
    t->drain();
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int flags)
{
    if (!e)
        return hipErrorInvalidValue;
    *e = new ihipEvent_t();
    (*e)->timing = !(flags & hipEventDisableTiming);
    return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t e)
{
    if (!e)
        return hipErrorInvalidValue;
    {
        // HIP lets an event be destroyed while its record is pending; the
        // stand-in waits for it, so that the record's work item stays valid
        std::unique_lock<std::mutex> lk(e->m);
        e->cv.wait(lk, [e] { return e->done >= e->recorded; });
    }
    delete e;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    if (!e)
        return hipErrorInvalidValue;
    ihipStream_t* t = resolve(s);
    if (t->capture) {
        std::lock_guard<std::mutex> lk(e->m);
        e->capture_id = t->capture->id;
        e->capture_stream = t;
        e->capture_seq = t->capture_seq;
        return hipSuccess;  // an ordering point inside the graph: nothing to run
    }
    uint64_t gen;
    {
        std::lock_guard<std::mutex> lk(e->m);
        e->capture_id = 0;
        gen = ++e->recorded;
    }
    t->push([e, gen] {
        {
            std::lock_guard<std::mutex> lk(e->m);
            e->done = std::max(e->done, gen);
            e->t = std::chrono::steady_clock::now();
        }
        e->cv.notify_all();
    });
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int)
{
    if (!e)
        return hipErrorInvalidValue;
    ihipStream_t* t = resolve(s);
    uint64_t cap, seq, gen;
    ihipStream_t* from;
    {
        std::lock_guard<std::mutex> lk(e->m);
        cap = e->capture_id;
        from = e->capture_stream;
        seq = e->capture_seq;
        gen = e->recorded;
    }
    if (cap) {
        std::lock_guard<std::mutex> lk(g_capture_m);
        auto it = g_open_captures.find(cap);
        if (it == g_open_captures.end())
            die("wait for an event recorded in a capture that has ended");
        ihipGraph* g = it->second;
        if (!t->capture) {  // t joins the capture
            t->capture = g;
            t->capture_seq = 0;
            g->joined[t] = {0, 0};
        } else if (t->capture != g) {
            die("stream waits for an event of another capture");
        }
        if (t == g->origin && from != g->origin) {
            auto& j = g->joined[from];
            j.second = std::max(j.second, seq);
        }
        return hipSuccess;
    }
    if (t->capture)
        die("a capturing stream waits for an event recorded outside the capture");
    t->push([e, gen] {
        std::unique_lock<std::mutex> lk(e->m);
        e->cv.wait(lk, [e, gen] { return e->done >= gen; });
    });
    return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t e)
{
    if (!e)
        return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(e->m);
    return e->done >= e->recorded ? hipSuccess : hipErrorNotReady;
}

hipError_t hipEventSynchronize(hipEvent_t e)
{
    if (!e)
        return hipErrorInvalidValue;
    std::unique_lock<std::mutex> lk(e->m);
    const uint64_t gen = e->recorded;
    e->cv.wait(lk, [e, gen] { return e->done >= gen; });
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b)
{
    if (!ms || !a || !b)
        return hipErrorInvalidValue;
    if (!a->timing || !b->timing)
        return hipErrorInvalidResourceHandle;
    std::lock_guard<std::mutex> la(a->m);
    std::lock_guard<std::mutex> lb(b->m);
    if (a->done < a->recorded || b->done < b->recorded || a->recorded == 0 || b->recorded == 0)
        return hipErrorNotReady;
    *ms = (float)std::chrono::duration<double, std::milli>(b->t - a->t).count();
    return hipSuccess;
}

hipError_t hipLaunchHostFunc(hipStream_t s, hipHostFn_t fn, void* user_data)
{
    if (!fn)
        return hipErrorInvalidValue;
    submit(resolve(s), [fn, user_data] { fn(user_data); });
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    ihipStream_t* t = resolve(s);
    if (t->capture)
        return hipErrorInvalidValue;
    ihipGraph* g = new ihipGraph();
    g->origin = t;
    {
        std::lock_guard<std::mutex> lk(g_capture_m);
        g->id = g_next_capture++;
        g_open_captures[g->id] = g;
    }
    t->capture = g;
    t->capture_seq = 0;
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* graph)
{
    ihipStream_t* t = resolve(s);
    ihipGraph* g = t->capture;
    if (!g || g->origin != t || !graph)
        return hipErrorInvalidValue;
    {
        std::lock_guard<std::mutex> lk(g_capture_m);
        g_open_captures.erase(g->id);
    }
    for (auto& kv : g->joined) {
        if (kv.second.second < kv.second.first)
            die("capture ended with a joined stream's work not joined back into the origin stream");
        kv.first->capture = nullptr;
    }
    t->capture = nullptr;
    g->open = false;
    *graph = g;
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t graph, hipGraphNode_t*, char*, size_t)
{
    if (!exec || !graph || graph->open)
        return hipErrorInvalidValue;
    hipGraphExec* x = new hipGraphExec();
    x->ops = graph->ops;
    *exec = x;
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s)
{
    if (!exec)
        return hipErrorInvalidValue;
    ihipStream_t* t = resolve(s);
    if (t->capture)
        die("graph launched into a capture");
    ++exec->queued;
    t->push([exec] {
        for (auto& f : exec->ops)
            f();
        --exec->queued;
    });
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t graph)
{
    if (!graph)
        return hipErrorInvalidValue;
    if (graph->open)
        die("graph destroyed while it is being captured");
    delete graph;
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t exec)
{
    if (!exec)
        return hipErrorInvalidValue;
    if (exec->queued.load() != 0)
        die("executable graph destroyed while a launch of it is queued or running");
    delete exec;
    return hipSuccess;
}

}  // extern "C++"

// Reported by the driver at exit: frees that had to wait for queued work.
uint64_t cpu_hip_free_waits() { return g_free_waits.load(); }

// The launches of batched rounds as they are issued (host order): for a wait,
// form is -1 and value the microseconds; for a batched sweep, form is the
// kernel form (muca_info::kernel_variant) and value L.
struct CpuHipLaunch {
    const void* stream;
    int form;
    uint32_t value;
};
namespace {
std::mutex g_log_m;
std::vector<CpuHipLaunch> g_log;
void log_launch(hipStream_t s, int form, uint32_t value)
{
    std::lock_guard<std::mutex> lk(g_log_m);
    g_log.push_back(CpuHipLaunch{s, form, value});
}
}  // namespace
std::vector<CpuHipLaunch> cpu_hip_take_launch_log()
{
    std::lock_guard<std::mutex> lk(g_log_m);
    std::vector<CpuHipLaunch> out;
    out.swap(g_log);
    return out;
}

// -- stand-in kernels -------------------------------------------------------

namespace muca {
namespace {

enum TableKind { kTableU64x4, kTableU32x5, kTableU32x8 };

size_t table_bytes(uint32_t N, TableKind k)
{
    return k == kTableU64x4 ? (size_t)(N + 1) * 4 * 8 : (size_t)(N + 1) * (k == kTableU32x5 ? 5 : 8) * 4;
}

bool reachable(uint32_t N, uint32_t k) { return k != 1 && k != N - 1; }

// Counts of the recorded sweeps [therm, nsweeps) of a launch that starts at
// instance sweep sweep0: each sweep of each live walker adds N counts, spread
// evenly over the first K reachable bins (the remainder in bin 0), with
// K = min(N + 1, 16 * 2^(sweep / 200)) for that sweep.  Per sweep, so that a
// run cut into launches counts exactly what one launch would.
void record(unsigned long long* hist, uint32_t N, uint64_t sweep0, uint32_t therm, uint32_t nsweeps, uint64_t live)
{
    for (uint32_t t = therm; t < nsweeps;) {
        const uint64_t sw = sweep0 + t;
        const uint64_t run = std::min<uint64_t>(nsweeps - t, (sw / 200 + 1) * 200 - sw);  // same K
        const uint64_t shift = std::min<uint64_t>(sw / 200, 24);
        const uint32_t K = (uint32_t)std::min<uint64_t>((uint64_t)N + 1, 16ull << shift);
        uint32_t bins = 0;
        for (uint32_t k = 0; k < K; ++k)
            bins += reachable(N, k);
        const uint64_t units = live * run;
        for (uint32_t k = 0; k < K; ++k)
            if (reachable(N, k))
                hist[k] += units * (N / bins);
        hist[0] += units * (N % bins);
        t += (uint32_t)run;
    }
}

// What one 64-walker block of a sweep kernel reads and writes, and its counts.
template <class A>
uint64_t run_block(uint32_t L, const A& a, uint32_t block, TableKind tk, bool may_idle, const char* who)
{
    const uint32_t N = L * L;
    if ((uint64_t)block * kWave >= a.wpad) {
        if (!may_idle)
            die(who);
        return 0;
    }
    if (a.wpad % kWave != 0 || a.walkers > a.wpad || a.walkers == 0)
        die("sweep arguments: walkers and padding do not agree");
    const size_t words = (size_t)L * words_per_row(L);
    check_range(a.spins, words * a.wpad * sizeof(uint32_t), kDevice, "sweep: lattice out of bounds");
    check_range(a.energy, (size_t)a.wpad * sizeof(int32_t), kDevice, "sweep: energies out of bounds");
    check_range(a.table, table_bytes(N, tk), kDevice, "sweep: threshold table out of bounds");
    check_range(a.hist, (size_t)(N + 1) * sizeof(uint64_t), kDevice, "sweep: histogram out of bounds");
    const uint32_t therm = std::min(a.therm, a.nsweeps);
    uint64_t live = 0;
    volatile uint32_t sink = 0;
    for (uint32_t lane = 0; lane < kWave; ++lane) {
        const uint32_t w = block * kWave + lane;
        for (size_t j = 0; j < words; ++j) {
            uint32_t& word = a.spins[j * a.wpad + w];
            word = word ^ 0u;
        }
        const int32_t E = a.energy[w];
        if (E < -2 * (int32_t)N || E > 2 * (int32_t)N || (E + 2 * (int32_t)N) % 4 != 0)
            die("sweep: energy out of range");
        a.energy[w] = E;
        live += w < a.walkers;
    }
    const uint8_t* t = reinterpret_cast<const uint8_t*>(a.table);
    sink = sink + t[0] + t[table_bytes(N, tk) - 1];
    record(a.hist, N, a.sweep0, therm, a.nsweeps, live);
    return (uint64_t)kWave * N * a.nsweeps;
}

template <class A>
void single(uint32_t L, const A& a, hipStream_t s, TableKind tk, uint32_t blocks_per_group, const char* who)
{
    const A c = a;
    submit(resolve(s), [L, c, tk, blocks_per_group, who] {
        const uint32_t blocks = c.wpad / kWave;
        uint64_t att = 0;
        for (uint32_t b = 0; b < blocks; ++b)
            att += run_block(L, c, b, tk, false, who);
        (void)blocks_per_group;
        simulate((double)att);
    });
}

template <class A>
void batch(uint32_t L, const A* args, const BatchItem* items, uint32_t nitems, hipStream_t s, TableKind tk,
           uint32_t blocks_per_item, bool may_idle, const char* who)
{
    check_range(items, (size_t)nitems * sizeof(BatchItem), kDevice, "batch: work items out of bounds");
    submit(resolve(s), [=] {
        check_range(items, (size_t)nitems * sizeof(BatchItem), kDevice, "batch: work items freed");
        uint64_t att = 0;
        for (uint32_t i = 0; i < nitems; ++i) {
            const BatchItem it = items[i];
            check_range(args + it.member, sizeof(A), kDevice, "batch: member arguments out of bounds");
            const A a = args[it.member];
            for (uint32_t g = 0; g < blocks_per_item; ++g)
                att += run_block(L, a, it.block * blocks_per_item + g, tk, may_idle || g > 0, who);
        }
        simulate((double)att);
    });
}

}  // namespace

bool sweep_supported(uint32_t L) { return L >= 4 && L % 2 == 0 && (L <= 64 || L == 80 || L == 96 || L == 112 || L == 128); }
bool fast_sweep_supported(uint32_t L) { return L >= 4 && L <= 64 && L % 2 == 0; }
bool split_sweep_supported(uint32_t L) { return fast_sweep_supported(L) && L != 62; }
bool pair_sweep_supported(uint32_t L) { return L == 48 || L == 52 || L == 56 || L == 64; }
bool wide_sweep_supported(uint32_t L) { return L == 80 || L == 96 || L == 112 || L == 128; }
bool wide_split_supported(uint32_t L) { return wide_sweep_supported(L); }

hipError_t launch_fast_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s)
{
    single(L, a, s, kTableU32x5, fast_waves_per_group(L), "one-wave sweep: block past the walkers");
    return hipSuccess;
}
hipError_t launch_split_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s)
{
    single(L, a, s, kTableU32x5, 1, "two-wave sweep: block past the walkers");
    return hipSuccess;
}
hipError_t launch_pair_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s)
{
    single(L, a, s, kTableU32x5, 2, "pair sweep: block past the walkers");
    return hipSuccess;
}
hipError_t launch_wide_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s)
{
    single(L, a, s, kTableU32x8, 1, "wide sweep: block past the walkers");
    return hipSuccess;
}
hipError_t launch_wide_split_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s)
{
    single(L, a, s, kTableU32x8, 1, "wide two-wave sweep: block past the walkers");
    return hipSuccess;
}
hipError_t launch_sweep(uint32_t L, const SweepArgs& a, hipStream_t s)
{
    single(L, a, s, kTableU64x4, 1, "generic sweep: block past the walkers");
    return hipSuccess;
}

hipError_t launch_init(const InitArgs& a, hipStream_t s)
{
    const InitArgs c = a;
    const size_t words = (size_t)a.L * words_per_row(a.L);
    check_range(a.spins, words * a.wpad * sizeof(uint32_t), kDevice, "init: lattice out of bounds");
    check_range(a.energy, (size_t)a.wpad * sizeof(int32_t), kDevice, "init: energies out of bounds");
    submit(resolve(s), [c, words] {
        std::memset(c.spins, 0, words * c.wpad * sizeof(uint32_t));  // all spins down: E = -2N
        for (uint32_t w = 0; w < c.wpad; ++w)
            c.energy[w] = -2 * (int32_t)(c.L * c.L);
    });
    return hipSuccess;
}

hipError_t launch_dispatch_delay(uint32_t microseconds, hipStream_t s)
{
    log_launch(s, -1, microseconds);
    if (microseconds)
        submit(resolve(s), [microseconds] {
            std::this_thread::sleep_for(std::chrono::microseconds(microseconds));
        });
    return hipSuccess;
}

hipError_t launch_fill_u64(unsigned long long* p, size_t n, hipStream_t s)
{
    check_range(p, n * sizeof(uint64_t), kDevice, "fill: out of bounds");
    submit(resolve(s), [p, n] {
        check_range(p, n * sizeof(uint64_t), kDevice, "fill ran after its buffer was freed");
        std::fill(p, p + n, 0ull);
    });
    return hipSuccess;
}

hipError_t launch_sweep_range(const RangeArgs& a, hipStream_t s)
{
    if (a.site_begin >= a.site_end)
        return hipSuccess;
    if (a.L < 4 || a.L > 128 || a.site_end > a.L * a.L || a.wpad % kWave != 0)
        return hipErrorInvalidValue;
    const RangeArgs c = a;
    submit(resolve(s), [c] {
        const uint32_t N = c.L * c.L;
        const TableKind tk = c.table_stride == 0 ? kTableU64x4 : (c.table_stride == 5 ? kTableU32x5 : kTableU32x8);
        check_range(c.table, table_bytes(N, tk), kDevice, "range sweep: table out of bounds");
        check_range(c.hist, (size_t)(N + 1) * sizeof(uint64_t), kDevice, "range sweep: histogram out of bounds");
        check_range(c.energy, (size_t)c.wpad * sizeof(int32_t), kDevice, "range sweep: energies out of bounds");
        const uint32_t from = std::max(c.site_begin, c.rec_begin);
        const uint64_t per = c.site_end > from ? c.site_end - from : 0;
        c.hist[0] += per * c.walkers;
        simulate((double)c.wpad * (c.site_end - c.site_begin));
    });
    return hipSuccess;
}

hipError_t launch_sweep_batch(uint32_t L, const SweepArgs* args, const BatchItem* items, uint32_t nitems,
                              hipStream_t s)
{
    log_launch(s, 0, L);
    batch(L, args, items, nitems, s, kTableU64x4, 1, false, "generic batch: block past the walkers");
    return hipSuccess;
}
hipError_t launch_fast_batch(uint32_t L, uint32_t G, const FastSweepArgs* args, const BatchItem* items,
                             uint32_t nitems, hipStream_t s)
{
    if (G != 1 && G != 2 && G != 4)
        return hipErrorInvalidValue;
    log_launch(s, 1, L);
    batch(L, args, items, nitems, s, kTableU32x5, G, false, "one-wave batch: first block past the walkers");
    return hipSuccess;
}
hipError_t launch_wide_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items, uint32_t nitems,
                             hipStream_t s)
{
    log_launch(s, 3, L);
    batch(L, args, items, nitems, s, kTableU32x8, 1, false, "wide batch: block past the walkers");
    return hipSuccess;
}
hipError_t launch_pair_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items, uint32_t nitems,
                             hipStream_t s)
{
    if (!pair_sweep_supported(L))
        return hipErrorInvalidValue;
    log_launch(s, 5, L);
    batch(L, args, items, nitems, s, kTableU32x5, 2, false, "pair batch: first block past the walkers");
    return hipSuccess;
}
hipError_t launch_split_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items, uint32_t nitems,
                              hipStream_t s)
{
    log_launch(s, 2, L);
    batch(L, args, items, nitems, s, kTableU32x5, 1, false, "two-wave batch: block past the walkers");
    return hipSuccess;
}
hipError_t launch_wide_split_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items,
                                   uint32_t nitems, hipStream_t s)
{
    log_launch(s, 4, L);
    batch(L, args, items, nitems, s, kTableU32x8, 1, false, "wide two-wave batch: block past the walkers");
    return hipSuccess;
}

}  // namespace muca
