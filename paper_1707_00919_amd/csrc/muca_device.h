// muca_device.h -- launch interface between the host runtime and the gfx950
// kernels of libmuca.  Internal: not part of the public C ABI (include/muca.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace muca {

// Device layout of one instance (all arrays in HBM):
//   spins   uint32 [L * WPR][wpad]  bit x%32 of word y*WPR + x/32 is site
//                                   (x, y); bit set = spin +1.  Word j of
//                                   walker w lives at j*wpad + w, so the 64
//                                   lanes of a wave touch 256 contiguous bytes.
//   energy  int32  [wpad]
//   hist    uint64 [N + 1]
//   table   uint64 [(N + 1) * 4]   thresholds of the four moves that change
//                                   the energy, slot s = m - (m > 2) for m =
//                                   number of neighbours anti-aligned with the
//                                   spin (m = 2 means dE = 0: always accepted).
// wpad = walkers rounded up to a multiple of 64; the padding walkers run
// like the others but never count into the histogram.
constexpr uint32_t kWave = 64;

struct SweepArgs {
    uint32_t* spins;
    int32_t* energy;
    const uint64_t* table;
    unsigned long long* hist;
    uint64_t sweep0;     // instance sweep counter at the first sweep of the launch
    uint32_t wpad;
    uint32_t walkers;
    uint32_t seed;
    uint32_t nsweeps;    // sweeps of this launch
    uint32_t therm;      // the first `therm` sweeps of the launch are not counted
    uint32_t pad;
};

// Arguments of the fast and split sweeps (L <= 64): table holds, for every bin k and
// every count m = 0..4 of anti-aligned neighbours, S = T - 1 of the move with
// energy change 8 - 4m at table[k*5 + 4 - m] (valid when no reachable T is 0).
struct FastSweepArgs {
    uint32_t* spins;
    int32_t* energy;
    const uint32_t* table;
    unsigned long long* hist;
    uint64_t sweep0;
    uint32_t wpad;
    uint32_t walkers;
    uint32_t seed;
    uint32_t nsweeps;
    uint32_t therm;
    uint32_t pad;
};

// One workgroup of a batched launch: block `block` (64 walkers) of batch
// member `member`; the member's arguments are args[member].
struct BatchItem {
    uint32_t member;
    uint32_t block;
};

// A batch member's arguments as a kernel's own.  They are read through the
// constant address space (the table of arguments does not change while the
// kernel runs): a pointer loaded from there is taken to point to global
// memory, where one read from generic memory would stay generic -- and
// generic (flat) accesses share the counter that tracks LDS loads, so that
// every wait for an LDS result would drain all of them -- and no store of the
// sweep can be taken to change the arguments.
template <class A>
__device__ __forceinline__ A member_args(const A* args, uint32_t member)
{
    using CA = const __attribute__((address_space(4))) A;
    const CA* c = (const CA*)args + member;
    A a;
    a.spins = c->spins;
    a.energy = c->energy;
    a.table = c->table;
    a.hist = c->hist;
    a.sweep0 = c->sweep0;
    a.wpad = c->wpad;
    a.walkers = c->walkers;
    a.seed = c->seed;
    a.nsweeps = c->nsweeps;
    a.therm = c->therm;
    a.pad = 0u;
    return a;
}

struct InitArgs {
    uint32_t* spins;
    int32_t* energy;
    uint32_t L;
    uint32_t wpad;
    uint32_t seed;
    uint32_t pad;
};

inline uint32_t words_per_row(uint32_t L) { return (L + 31u) / 32u; }
inline uint32_t padded_walkers(uint32_t walkers) { return (walkers + kWave - 1) / kWave * kWave; }

// LDS an MI355X compute unit offers to the workgroups resident on it.
constexpr uint32_t kLdsPerCu = 160u * 1024u;

// LDS bytes of one workgroup of the fast sweep (a 28-byte record per energy
// bin).
__host__ __device__ constexpr uint32_t fast_lds_bytes(uint32_t L) { return 28u * (L * L + 1u); }

// The two-wave sweep's LDS: the records (28 bytes per energy bin; in the wide
// form, L > 64, the 32-bit counters alone), rounded up to 16 bytes so that the
// ring's 16-byte accesses are aligned, in front of a two-slot ring holding the
// Philox words of one loop step of `rows` rows per slot (16 bytes per block of
// four sites per walker).
__host__ __device__ constexpr uint32_t split_lds_bytes_for(uint32_t L, bool wide, uint32_t rows)
{
    return ((wide ? 4u : 28u) * (L * L + 1u) + 15u) / 16u * 16u + 2u * (rows * L / 4u) * (uint32_t)kWave * 16u;
}

// Two-wave workgroups one CU runs at once (at most two count: a third one's
// producer wave would compete with the chains).
__host__ __device__ constexpr uint32_t split_groups_per_cu(uint32_t bytes)
{
    return bytes > kLdsPerCu ? 0u : (kLdsPerCu / bytes < 2u ? kLdsPerCu / bytes : 2u);
}

// Rows per loop step of the two-wave sweep.  A step is whole rows of whole
// Philox blocks (one row when L is a multiple of 4, else two); it takes two or
// four times that many rows, up to 128 sites, where the longer ring slots still
// leave as many workgroups per CU.  Each step ends in a barrier and in loop
// bookkeeping on the chain wave, so longer steps shorten the chain.
__host__ __device__ constexpr uint32_t split_rows_per_step(uint32_t L, bool wide)
{
    const uint32_t base = L % 4u == 0u ? 1u : 2u;
    const uint32_t fit = split_groups_per_cu(split_lds_bytes_for(L, wide, base));
    uint32_t rows = base;
    for (uint32_t r = 2u * base; r <= 4u; r *= 2u)
        if (L % r == 0u && r * L <= 128u && split_groups_per_cu(split_lds_bytes_for(L, wide, r)) >= fit)
            rows = r;
    return rows;
}

// The pair form of the two-wave sweep: two chain waves of 64 walkers share one
// record table, each with a producer wave and a ring of its own, so that a CU
// whose LDS holds one table runs two chains.  A loop step is a row, or half a
// row where two rings of two row-long slots would not fit beside the table
// (L = 64); 0 where neither fits or a half row is not whole Philox blocks.
__host__ __device__ constexpr uint32_t pair_lds_bytes_for(uint32_t L, uint32_t sites)
{
    return (28u * (L * L + 1u) + 15u) / 16u * 16u + 2u * 2u * (sites / 4u) * (uint32_t)kWave * 16u;
}
__host__ __device__ constexpr uint32_t pair_sites_per_step(uint32_t L)
{
    return L % 4u != 0u || L > 64u ? 0u
           : pair_lds_bytes_for(L, L) <= kLdsPerCu ? L
           : (L % 8u == 0u && pair_lds_bytes_for(L, L / 2u) <= kLdsPerCu) ? L / 2u
                                                                          : 0u;
}
__host__ __device__ constexpr uint32_t pair_lds_bytes(uint32_t L) { return pair_lds_bytes_for(L, pair_sites_per_step(L)); }

// LDS bytes of one workgroup of the split sweep (L <= 64) and of the wide
// two-wave sweep (L > 64).
__host__ __device__ constexpr uint32_t split_lds_bytes(uint32_t L)
{
    return split_lds_bytes_for(L, false, split_rows_per_step(L, false));
}
__host__ __device__ constexpr uint32_t wide_split_lds_bytes(uint32_t L)
{
    return split_lds_bytes_for(L, true, split_rows_per_step(L, true));
}

// Waves (of 64 walkers each) per workgroup of the fast sweep.  The record
// table is per workgroup; where it is so large that fewer than four
// workgroups fit in a CU's LDS, several waves share one copy so that every
// SIMD of the CU still gets a chain to run.
__host__ __device__ constexpr uint32_t fast_waves_per_group(uint32_t L)
{
    return kLdsPerCu / fast_lds_bytes(L) >= 4u ? 1u : (kLdsPerCu / fast_lds_bytes(L) >= 2u ? 2u : 4u);
}

// The two-wave (split) form pays while every one of its workgroups is resident
// at once and at most two share a CU (their producer waves then do not compete
// with the chains); otherwise the one-wave form runs more chains at a time.
inline bool prefer_two_waves(uint32_t lds_bytes, uint64_t blocks, uint32_t cus)
{
    const uint64_t per_cu = kLdsPerCu / lds_bytes;
    return blocks <= (uint64_t)cus * (per_cu < 2u ? per_cu : 2u);
}
inline bool prefer_split(uint32_t L, uint64_t blocks, uint32_t cus)
{
    return prefer_two_waves(split_lds_bytes(L), blocks, cus);
}
inline bool prefer_wide_split(uint32_t L, uint64_t blocks, uint32_t cus)
{
    return prefer_two_waves(wide_split_lds_bytes(L), blocks, cus);
}
// Where one two-wave workgroup per CU is all that fits and there are more
// 64-walker blocks than CUs, the pair form runs two chains per CU: it pays
// while all of its workgroups are resident at once.
bool pair_sweep_supported(uint32_t L);
inline bool prefer_pair(uint32_t L, uint64_t blocks, uint32_t cus)
{
    return pair_sweep_supported(L) && split_groups_per_cu(split_lds_bytes(L)) == 1u && blocks > cus &&
           (blocks + 1u) / 2u <= (uint64_t)cus * split_groups_per_cu(pair_lds_bytes(L));
}

// Largest number of recorded sweeps one launch may run without a 32-bit LDS
// histogram counter overflowing: every walker of a workgroup (64 per wave,
// waves_per_group waves; by default fast_waves_per_group(L)) adds N counts
// per sweep to the same table.
inline uint32_t max_sweeps_per_launch(uint32_t L, uint32_t waves_per_group = 0)
{
    const uint32_t G = waves_per_group ? waves_per_group : fast_waves_per_group(L);
    const uint64_t per_sweep = (uint64_t)kWave * G * L * L;
    const uint64_t m = 0xffffffffull / per_sweep;
    return m > 0x7fffffffull ? 0x7fffffffu : (uint32_t)m;
}

bool sweep_supported(uint32_t L);
bool fast_sweep_supported(uint32_t L);
hipError_t launch_fast_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s);
bool split_sweep_supported(uint32_t L);
hipError_t launch_split_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s);
// The pair form: one workgroup of four waves per two 64-walker blocks.
hipError_t launch_pair_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s);
hipError_t launch_init(const InitArgs& a, hipStream_t s);
// L > 64 with the thresholds in global memory: table holds, per bin k, S =
// T - 1 of the move with m anti-aligned neighbours at table[k*8 + 4 - m]
// (32-byte records; valid when no reachable T is 0).
bool wide_sweep_supported(uint32_t L);
hipError_t launch_wide_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s);
// The same tables with the random numbers on a second wave (two-wave form).
bool wide_split_supported(uint32_t L);
hipError_t launch_wide_split_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s);
hipError_t launch_sweep(uint32_t L, const SweepArgs& a, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, size_t n, hipStream_t s);

// Arguments of a partial sweep: sites [site_begin, site_end) of one sweep, in
// typewriter order, the sites from rec_begin on counted in the histogram.
// table is in the generic layout (uint64, 4 per bin; table_stride 0) or holds
// uint32 S = T - 1 by 4 - m, table_stride words per bin (5, or 8 for L > 64).
struct RangeArgs {
    uint32_t* spins;
    int32_t* energy;
    const void* table;
    unsigned long long* hist;
    uint64_t sweep;
    uint32_t L, wpad, walkers, seed;
    uint32_t site_begin, site_end, rec_begin;
    uint32_t table_stride;
};
hipError_t launch_sweep_range(const RangeArgs& a, hipStream_t s);

// Batched forms: one launch runs nitems workgroups, each described by
// items[i], all members of the batch having the same L.
hipError_t launch_sweep_batch(uint32_t L, const SweepArgs* args, const BatchItem* items,
                              uint32_t nitems, hipStream_t s);
// One-wave form with G (1, 2 or 4) waves of 64 walkers per workgroup.
hipError_t launch_fast_batch(uint32_t L, uint32_t G, const FastSweepArgs* args, const BatchItem* items,
                             uint32_t nitems, hipStream_t s);
hipError_t launch_wide_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items, uint32_t nitems,
                             hipStream_t s);
// Pair-form work items: BatchItem::block is the pair's index (blocks 2i, 2i+1).
hipError_t launch_pair_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items, uint32_t nitems,
                             hipStream_t s);
hipError_t launch_split_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items,
                              uint32_t nitems, hipStream_t s);
hipError_t launch_wide_split_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items,
                                   uint32_t nitems, hipStream_t s);

}  // namespace muca
