// muca_internal.h -- host-side state shared by the instance runtime and the
// batched runtime of libmuca.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "muca.h"
#include "muca_host_math.h"

namespace muca {
// A wait of about `microseconds` on stream s, in front of a batched round's
// one-wave launches so that its two-wave launches are dispatched first
// (muca_order.hip).
hipError_t launch_dispatch_delay(uint32_t microseconds, hipStream_t s);
}  // namespace muca

namespace muca_host {

struct Layout {
    size_t spins_off, spins_bytes;
    size_t energy_off, energy_bytes;
    size_t hist_off, hist_bytes;
    size_t table_off, table_bytes;
    size_t total;
};


}  // namespace muca_host

struct muca_instance {
    muca_params p{};
    uint32_t L = 0, N = 0, wpr = 0, wpad = 0;
    int device = 0;
    int cus = 256;  // compute units of the device
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* ws = nullptr;
    bool own_ws = false;
    muca_host::Layout lay{};
    uint32_t* d_spins = nullptr;
    int32_t* d_energy = nullptr;
    unsigned long long* d_hist = nullptr;
    uint64_t* d_table = nullptr;
    uint64_t* h_table4 = nullptr;  // pinned staging for the device table
    uint64_t* h_hist = nullptr;    // pinned staging for the histogram
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    std::vector<double> omega;
    std::vector<uint64_t> table5;  // thresholds of the last sweep call
    std::vector<uint64_t> hist;    // histogram of the last recorded call
    uint64_t position = 0;  // attempts made per walker so far (sweep = position / N)
    uint32_t iteration = 0;
    int width_prev = 0;  // covered range of the last recorded call, in bins
    int reach_prev = 0;  // reachable bins inside it
    muca_info last{};
    bool poisoned = false;
    std::string err;
};


namespace muca_host {

// Device buffers and shape of one sweep call (an instance's, or those the
// caller of the allocation-free production call hands in).
struct CallTarget {
    uint32_t L, wpad, walkers, seed, flags;
    int cus;
    uint32_t* d_spins;
    int32_t* d_energy;
    unsigned long long* d_hist;  // N + 1 bins
    uint64_t* d_table;           // 32 (N + 1) bytes
    uint64_t* h_table4;          // host staging of the device table, same size
};

// Picks the kernel form for the thresholds table5 (T[k*5 + d]), writes the
// device form of the table into t.h_table4 and enqueues on `stream`: its
// upload, the histogram clear and the launches of every segment (between
// ev_start and ev_stop when they are not null).  Nothing is waited for.
// Returns the first failing HIP call's error, *what naming it.
hipError_t enqueue_call(const CallTarget& t, const uint64_t* table5, const Segment* segs, size_t nsegs,
                        hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_stop, uint32_t* launches,
                        uint32_t* variant, const char** what);

// Sets the message muca_last_error(NULL) returns on this thread (copied into
// a fixed buffer; never allocates).
void set_null_error(const char* msg);

// Apply the results of a finished recorded call (histogram already in
// h->hist): checks sum H, fills the statistics, applies Eq. 4 when `update`.
// Returns MUCA_OK or an error code (the instance is then poisoned).
int finish_call(muca_instance* h, uint64_t therm, uint64_t recorded, bool update, double kernel_ms,
                uint32_t launches, uint32_t variant, muca_info* info);

}  // namespace muca_host
