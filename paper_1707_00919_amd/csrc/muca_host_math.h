// muca_host_math.h -- host arithmetic of libmuca that needs no device (see
// muca_host_math.cpp).  Not part of the public C ABI; plain C++, no HIP.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <iterator>
#include <map>
#include <vector>

namespace muca_host {

// Acceptance thresholds T[k*5+d] from the log weights (IEEE double, libm exp).
void compute_thresholds(uint32_t N, const double* om, uint64_t* t5);
// Generic-kernel table: uint64 thresholds of the four energy-changing moves.
void device_table(uint32_t N, const uint64_t* t5, uint64_t* t4);
// Table of the fast, split and wide kernels: uint32 S = T - 1 at
// f[k*stride + 4 - m] by the number m of anti-aligned neighbours, i.e. at
// slot 2 + d for the bin change d = 2 - m of the move (stride 5, or 8 for the
// wide kernel's 32-byte records, the rest zero); false if a move that can be
// proposed has T = 0.
bool fast_table(uint32_t N, const uint64_t* t5, uint32_t* f, uint32_t stride);
double flatness_of(uint32_t N, const uint64_t* H);
double chebyshev_of(uint32_t N, const uint64_t* H);
// ln g[k] = ln H[k] - omega[k] + c on reachable bins with H > 0, -inf
// elsewhere; normalization 0: ln g[0] = ln 2, 1: sum exp(ln g) = 2^N.
// Returns 0, or 1 (ground-state bin empty) / 2 (histogram empty).
int log_dos_of(uint32_t N, const uint64_t* H, const double* omega, int normalization, double* out);
// Eq. 6 with Q uniform over max(reach_prev, 10) bins.
double kl_of(uint32_t N, const uint64_t* H, int reach_prev);
// Reachable bins (not 1 or N-1) between the lowest and highest visited bin.
int reach_of(uint32_t N, const uint64_t* H);
int width_of(uint32_t N, const uint64_t* H);

// One piece of a call: whole sweeps [sweep0, sweep0 + n) of which the first
// `therm` are not recorded, or (n == 0) the sites [site_begin, site_end) of
// sweep sweep0 with recording from site rec_begin on.
struct Segment {
    uint64_t sweep0;
    uint64_t n;
    uint64_t therm;
    uint32_t site_begin, site_end, rec_begin;
};

// Cuts the attempts [pos0, pos0 + therm + recorded) -- recording from
// pos0 + therm on -- into whole-sweep runs for the sweep kernels and partial
// sweeps for the range kernel.
std::vector<Segment> segments_of(uint64_t N, uint64_t pos0, uint64_t therm, uint64_t recorded);

// Launch planning of one batched round (no device involved).  Forms are
// numbered as muca_info::kernel_variant: 0 generic, 1 one-wave (fast), 2
// two-wave (split), 3 wide one-wave, 4 wide two-wave, 5 two-wave pairs.
enum : uint32_t { kFormGeneric = 0, kFormFast = 1, kFormSplit = 2, kFormWide = 3, kFormWideSplit = 4, kFormPair = 5 };
// Launch shapes: two-wave for all, one-wave with default wave groups, one-wave
// with four waves per table, mixed (the longest chains first, as many as fit),
// mixed-longest (only the members whose chain is the round's longest).
enum : int { kShapeTwoWave = 0, kShapeOneWave = 1, kShapeOneWaveFour = 2, kShapeMixed = 4, kShapeMixedLongest = 5 };

// One member of a round as the planner sees it.  table: the table the member's
// weights allow this round -- kFormFast (the LDS-record kernels), kFormWide or
// kFormGeneric.
struct RoundMember {
    bool active = false;        // not skipped this round
    uint32_t L = 0;
    uint32_t blocks = 0;        // 64-walker blocks
    uint32_t walkers = 0;
    uint64_t chain = 0;         // attempts one walker makes this round
    uint32_t table = kFormGeneric;
    bool forced_fast = false;   // MUCA_FLAG_FAST_KERNEL
    bool split_ok = false, fast_ok = false, pair_ok = false, wide_split_ok = false;
    uint32_t two_wave_bytes = 0;   // LDS of one two-wave workgroup (split or wide split), 0: none
    uint32_t fast_waves = 1;       // waves per workgroup of the one-wave form by default
};

// Whether a round's two-wave workgroups all fit on the device at once, at
// most two chains per CU (LDS shares weighted by each L): with one workgroup
// per chain (single), or with pairs for the members whose split workgroup
// fills a CU (pairable).  share[i]: member i's share of the CUs in the
// arrangement used (pairs wherever single does not fit); 0 if it has no
// two-wave form.
struct RoundFit {
    bool two_wave_single = false;
    bool two_wave = false;
    bool use_pairs = false;
    uint64_t walkers = 0;
    std::vector<double> share;
    std::vector<char> pairable;
};
RoundFit round_fit(const RoundMember* m, size_t n, uint32_t cus, uint32_t lds_per_cu);

// Forms and waves per workgroup of every member for a launch shape; in the
// mixed shape the two-wave form goes to the members with the longest chains
// (then the fewest walkers) while their shares fit, in the mixed-longest
// shape only to those whose chain equals the round's longest.
void plan_forms(const RoundMember* m, size_t n, uint32_t cus, const RoundFit& fit, int shape, uint32_t* form,
                uint32_t* waves);

// Estimated attempts of one served solve: walkers * N per sweep, times the
// sweeps it asks for -- its weight iterations of iter_therm + iter_sweeps
// sweeps each, then prod_therm + prod_sweeps.  The number of iterations to a
// flat histogram is taken to grow like N (about N / 20: 48 at L = 32 with
// 16384 walkers and 200-sweep iterations), capped by max_iterations when that
// is set.
double solve_work_estimate(uint32_t L, uint32_t walkers, uint32_t iter_therm, uint32_t iter_sweeps,
                           uint32_t max_iterations, uint32_t prod_therm, uint32_t prod_sweeps);

// The serving queue's admission order.  Entries are in arrival order.  FIFO
// (smallest_first false) takes entry 0.  Smallest-first takes the entry of
// least work (ties: the earlier arrival) -- unless some entry has waited
// longer than max_wait_s at time now, in which case the oldest such entry
// goes first, so that no request waits without bound behind a stream of
// smaller ones.
struct QueuedJob {
    double work;
    double t_submit;
};
size_t admission_pick(const QueuedJob* q, size_t n, bool smallest_first, double now, double max_wait_s);

constexpr size_t kArenaAlign = 256;

// First-fit allocator over [0, size) with coalescing of free neighbours: the
// serving form carves every admitted request's device state out of one arena.
// Sizes are rounded up to kArenaAlign bytes; release takes what alloc gave.
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size)
            free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    bool alloc(size_t n, size_t* off)
    {
        n = (n + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t at = it->first + n;
                free_.erase(it);
                if (rest)
                    free_[at] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
        used_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size_ = 0, used_ = 0;
};

}  // namespace muca_host
