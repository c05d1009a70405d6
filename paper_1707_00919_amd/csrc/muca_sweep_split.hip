// muca_sweep_split.hip -- the multicanonical sweep with the random numbers and
// the Metropolis chain on two different waves (gfx950).
//
// Each walker's chain is serial: an attempt's threshold depends on the energy
// the previous attempt left behind (Sec. 2.2-2.3).  With 64 walkers per wave
// and a few thousand walkers per GPU, one wave per SIMD is all there is, so the
// chain's latency, not the chip's issue rate, sets the pace.  This kernel
// shortens it in two ways:
//
//  * A workgroup has two waves for the same 64 walkers.  The producer wave
//    runs Philox4x32-10 for the next loop step (one to four rows, or half a
//    row in the pair form at L = 64) and writes the words to an LDS ring; the
//    consumer wave runs only the chain, reading four draws with one 16-byte
//    LDS load.  One barrier per loop step hands a ring slot over.
//  * The consumer's chain step (muca_chain.h) resolves attempt x while the two
//    thresholds attempt x+1 can need are already on their way.
//
// The pair form (L = 48..64, where one such workgroup fills a CU's LDS) puts
// two chain waves and their two producer waves in one workgroup around one
// record table, so that a CU runs two chains.
//
// For L <= 64 the per-bin records live in LDS: 28 bytes (7 words: the five
// thresholds S = T - 1 by the number m of anti-aligned neighbours, from m = 4
// down, the histogram counter, one pad word); an odd word stride spreads the
// gathers of 64 lanes over all banks.  For L = 80..128 (the wide form) the
// records do not fit: the chain reads the 32-byte threshold records from
// global memory through the caches and LDS holds only the 32-bit counters in
// front of the ring.  The row bookkeeping (site words) is in muca_rowbits.h.
#include <type_traits>

#include "muca_device.h"

#include "muca_chain.h"
#include "philox.h"

namespace muca {
namespace {

// A workgroup of CHAINS chain waves and as many producer waves.  Loop steps
// of SPS sites: split_rows_per_step(L, WIDE) rows for the one-chain form,
// pair_sites_per_step(L) (a row or half a row) for the pair form.  LDS: the
// records (or, in the wide form, the counters) in front of a two-slot ring
// per chain, each slot one loop step; slots start on a 16-byte boundary so
// that every 16-byte ring access is aligned.
template <int L, bool WIDE, int CHAINS>
struct SplitShape : ChainShape<L> {
    using C = ChainShape<L>;
    static_assert(CHAINS == 1 || (CHAINS == 2 && !WIDE), "the pair form is for L <= 64");
    static constexpr int SPS = CHAINS == 1 ? (int)split_rows_per_step(L, WIDE) * L : (int)pair_sites_per_step(L);
    static_assert(SPS > 0 && SPS % 4 == 0 && (SPS % L == 0 || (SPS * 2 == L)),
                  "a loop step is whole rows, or half a row, of whole Philox blocks");
    static constexpr int RPS = SPS >= L ? SPS / L : 0;  // 0: half-row steps
    static constexpr int STEPS = C::N / SPS;           // per sweep
    static constexpr int BLOCKS = SPS / 4;
    static constexpr int FRONT_BYTES = ((WIDE ? 4 * (C::N + 1) : C::REC_BYTES) + 15) / 16 * 16;
    static constexpr int SLOT_BYTES = BLOCKS * kWave * 16;
    static constexpr int RING_BYTES = 2 * SLOT_BYTES;
    static constexpr int LDS_BYTES = FRONT_BYTES + CHAINS * RING_BYTES;
};

// The consumer's random words: one 16-byte load per block from the ring slot
// the producer filled for this loop step.
struct RingDraws {
    const uint8_t* lds;
    uint32_t slot;
    uint32_t lane;
    template <int B>
    __device__ __forceinline__ Words4 block() const
    {
        const uint4 v = *reinterpret_cast<const uint4*>(lds + slot + (uint32_t)(B * kWave + lane) * 16u);
        return Words4{{v.x, v.y, v.z, v.w}};
    }
    __device__ __forceinline__ Words4 first() const { return block<0>(); }
    template <int B, int PART>
    __device__ __forceinline__ void advance(Words4& rn)
    {
        if constexpr (PART == 0)
            rn = block<B>();
    }
};

// Producer: the Philox words of every site of loop step s into slot s & 1 of
// the ring at byte `ring`.
template <class S>
__device__ __forceinline__ void produce_step(uint8_t* lds, uint32_t ring, uint32_t s, const FastSweepArgs& a,
                                             uint32_t walker, uint32_t lane)
{
    const uint32_t t = s / S::STEPS;
    const uint64_t sweep = a.sweep0 + t;
    const uint32_t blk0 = (s - t * S::STEPS) * (uint32_t)S::BLOCKS;
    uint8_t* slot = lds + ring + (s & 1u) * S::SLOT_BYTES;
#pragma unroll 2
    for (int b = 0; b < S::BLOCKS; ++b) {
        const Words4 r = philox10(blk0 + (uint32_t)b, (uint32_t)sweep, (uint32_t)(sweep >> 32), 0u,
                                  a.seed, walker);
        *reinterpret_cast<uint4*>(slot + (uint32_t)(b * kWave + lane) * 16u) =
            uint4{r.w[0], r.w[1], r.w[2], r.w[3]};
    }
}

// One workgroup: chain waves 0 .. CHAINS-1 run the chains of 64-walker
// blocks group * CHAINS + c; producer wave CHAINS + c fills chain c's ring.
// A pair whose second block is past the instance's walkers leaves that
// chain and its producer idle (they still take part in every barrier).
template <int L, bool WIDE, int CHAINS>
__device__ __forceinline__ void sweep_split_kernel_body(const FastSweepArgs& a, uint32_t group)
{
    using S = SplitShape<L, WIDE, CHAINS>;
    using R = std::conditional_t<WIDE, GlobalRecords, LdsRecords>;
    constexpr int N = S::N;
    constexpr int THREADS = 2 * CHAINS * kWave;
    static_assert(S::LDS_BYTES <= 160 * 1024, "records and rings must fit in LDS");
    static_assert(S::LDS_BYTES == (int)(CHAINS == 2 ? pair_lds_bytes(L)
                                        : WIDE    ? wide_split_lds_bytes(L)
                                                  : split_lds_bytes(L)),
                  "LDS size formula");
    __shared__ __attribute__((aligned(16))) uint8_t lds[S::LDS_BYTES];
    uint32_t* const counters = reinterpret_cast<uint32_t*>(lds);  // wide form

    const uint32_t lane = threadIdx.x & (kWave - 1);
    // The wave's role is made wave-uniform so that each wave takes one branch
    // as a whole and the loops' step arithmetic stays scalar.
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x) / kWave;
    const bool consumer = wave < (uint32_t)CHAINS;
    const uint32_t chain = consumer ? wave : wave - (uint32_t)CHAINS;
    const uint32_t block = group * (uint32_t)CHAINS + chain;
    const bool has = block * kWave < a.wpad;
    const uint32_t ring = S::FRONT_BYTES + chain * S::RING_BYTES;
    const uint32_t w = block * kWave + lane;
    const uint32_t steps = a.nsweeps * (uint32_t)S::STEPS;

    if constexpr (WIDE) {
        for (int k = threadIdx.x; k <= N; k += THREADS)
            counters[k] = 0u;
    } else {
        chain_records_fill<L>(lds, a.table, threadIdx.x, THREADS);
    }
    if (!consumer && has && steps > 0)
        produce_step<S>(lds, ring, 0u, a, w, lane);
    __syncthreads();

    // Each wave runs a loop of its own, with one barrier per loop step in
    // all: a loop shared by the waves would merge their paths every step and
    // carry the chain's state across in register copies.
    if (consumer && has) {
        uint32_t* const mine = a.spins + w;
        const size_t stride = a.wpad;
        ChainState<L> st;
        const uint32_t live = w < a.walkers ? 1u : 0u;
        R recs;
        if constexpr (WIDE)
            recs = GlobalRecords{reinterpret_cast<const uint8_t*>(a.table) + 8, lds};
        else
            recs = LdsRecords{lds};
        chain_load<L, R>(st, mine, stride, a.energy[w]);
        chain_prime<L>(st, recs);
        if constexpr (S::RPS > 0) {
            for (uint32_t s = 0; s < steps; ++s) {
                const uint32_t t = s / S::STEPS;
                const int y = (int)(s - t * S::STEPS) * S::RPS;
                const uint32_t inc = t >= a.therm ? live : 0u;
                RingDraws draws{lds, ring + (s & 1u) * S::SLOT_BYTES, lane};
                Words4 rn = draws.first();
                Words4 rc;
                chain_rows<L, S::RPS>(st, rc, rn, draws, recs, inc, mine, stride, y);
                __syncthreads();
            }
        } else {
            // half-row steps: a row is two steps, slots s & 1 and (s + 1) & 1
            for (uint32_t s = 0; s < steps; s += 2) {
                const uint32_t t = s / S::STEPS;
                const uint32_t y = (s - t * S::STEPS) / 2u;
                const uint32_t inc = t >= a.therm ? live : 0u;
                Words4 rc;
                chain_row_open<L>(st, recs, mine, stride, y);
                {
                    RingDraws draws{lds, ring + (s & 1u) * S::SLOT_BYTES, lane};
                    Words4 rn = draws.first();
                    chain_row_part<L, 0, L / 2>(st, rc, rn, draws, recs, inc);
                }
                __syncthreads();
                {
                    RingDraws draws{lds, ring + ((s + 1u) & 1u) * S::SLOT_BYTES, lane};
                    Words4 rn = draws.first();
                    chain_row_part<L, L / 2, L / 2>(st, rc, rn, draws, recs, inc);
                }
                chain_row_close<L>(st, mine, stride, y);
                __syncthreads();
            }
        }
        a.energy[w] = chain_finish<L>(st, recs);
    } else {
        const bool produce = !consumer && has;
        for (uint32_t s = 0; s < steps; ++s) {
            if (produce && s + 1 < steps)
                produce_step<S>(lds, ring, s + 1, a, w, lane);
            __syncthreads();
        }
    }
    __syncthreads();
    if constexpr (WIDE) {
        for (int k = threadIdx.x; k <= N; k += THREADS) {
            const uint32_t v = counters[k];
            if (v)
                atomicAdd(a.hist + k, (unsigned long long)v);
        }
    } else {
        chain_records_flush<L>(lds, a.hist, threadIdx.x, THREADS);
    }
}

template <int L>
__global__ __launch_bounds__(128) void sweep_split_kernel(FastSweepArgs a)
{
    sweep_split_kernel_body<L, false, 1>(a, blockIdx.x);
}

template <int L>
__global__ __launch_bounds__(128) void sweep_wide_split_kernel(FastSweepArgs a)
{
    sweep_split_kernel_body<L, true, 1>(a, blockIdx.x);
}

template <int L>
__global__ __launch_bounds__(256) void sweep_pair_kernel(FastSweepArgs a)
{
    sweep_split_kernel_body<L, false, 2>(a, blockIdx.x);
}

template <int L>
__global__ __launch_bounds__(128) void sweep_split_kernel_batch(const FastSweepArgs* args, const BatchItem* items)
{
    const BatchItem it = items[blockIdx.x];
    sweep_split_kernel_body<L, false, 1>(member_args(args, it.member), it.block);
}

template <int L>
__global__ __launch_bounds__(128) void sweep_wide_split_kernel_batch(const FastSweepArgs* args,
                                                                     const BatchItem* items)
{
    const BatchItem it = items[blockIdx.x];
    sweep_split_kernel_body<L, true, 1>(member_args(args, it.member), it.block);
}

template <int L>
__global__ __launch_bounds__(256) void sweep_pair_kernel_batch(const FastSweepArgs* args, const BatchItem* items)
{
    const BatchItem it = items[blockIdx.x];
    sweep_split_kernel_body<L, false, 2>(member_args(args, it.member), it.block);
}

template <int L>
hipError_t launch_pair_L(const FastSweepArgs& a, hipStream_t s)
{
    const uint32_t blocks = a.wpad / kWave;
    hipLaunchKernelGGL(sweep_pair_kernel<L>, dim3((blocks + 1u) / 2u), dim3(4 * kWave), 0, s, a);
    return hipGetLastError();
}

template <int L>
hipError_t launch_pair_L_batch(const FastSweepArgs* args, const BatchItem* items, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_pair_kernel_batch<L>, dim3(n), dim3(4 * kWave), 0, s, args, items);
    return hipGetLastError();
}

template <int L>
hipError_t launch_split_L_batch_L(const FastSweepArgs* args, const BatchItem* items, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_split_kernel_batch<L>, dim3(n), dim3(2 * kWave), 0, s, args, items);
    return hipGetLastError();
}

template <int L>
hipError_t launch_wide_split_L_batch(const FastSweepArgs* args, const BatchItem* items, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_wide_split_kernel_batch<L>, dim3(n), dim3(2 * kWave), 0, s, args, items);
    return hipGetLastError();
}

template <int L>
hipError_t launch_split_L(const FastSweepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_split_kernel<L>, dim3(a.wpad / kWave), dim3(2 * kWave), 0, s, a);
    return hipGetLastError();
}

template <int L>
hipError_t launch_wide_split_L(const FastSweepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_wide_split_kernel<L>, dim3(a.wpad / kWave), dim3(2 * kWave), 0, s, a);
    return hipGetLastError();
}

}  // namespace

// L = 62 is absent: its two-row ring slots and records overflow the 160 KiB
// of LDS (the fast kernel serves it).
#define MUCA_SPLIT_L(X)                                                                    \
    X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(26) X(28) X(30) X(32) \
    X(34) X(36) X(38) X(40) X(42) X(44) X(46) X(48) X(50) X(52) X(54) X(56) X(58) X(60)    \
    X(64)

bool split_sweep_supported(uint32_t L)
{
    switch (L) {
#define MUCA_CASE(LL) case LL:
        MUCA_SPLIT_L(MUCA_CASE)
#undef MUCA_CASE
        return true;
    default:
        return false;
    }
}

hipError_t launch_split_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s)
{
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_split_L<LL>(a, s);
        MUCA_SPLIT_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

// The pair form where one two-wave workgroup fills a CU's LDS and two rings
// of whole rows, or of half rows, fit beside the table (not L = 60: its half
// rows are not whole Philox blocks).
#define MUCA_PAIR_L(X) X(48) X(52) X(56) X(64)

bool pair_sweep_supported(uint32_t L)
{
    switch (L) {
#define MUCA_CASE(LL) case LL:
        MUCA_PAIR_L(MUCA_CASE)
#undef MUCA_CASE
        return true;
    default:
        return false;
    }
}

hipError_t launch_pair_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s)
{
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_pair_L<LL>(a, s);
        MUCA_PAIR_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_pair_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items, uint32_t nitems,
                             hipStream_t s)
{
    if (nitems == 0)
        return hipSuccess;
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_pair_L_batch<LL>(args, items, nitems, s);
        MUCA_PAIR_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

#define MUCA_WIDE_SPLIT_L(X) X(80) X(96) X(112) X(128)

bool wide_split_supported(uint32_t L)
{
    switch (L) {
#define MUCA_CASE(LL) case LL:
        MUCA_WIDE_SPLIT_L(MUCA_CASE)
#undef MUCA_CASE
        return true;
    default:
        return false;
    }
}

hipError_t launch_wide_split_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s)
{
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_wide_split_L<LL>(a, s);
        MUCA_WIDE_SPLIT_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_wide_split_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items, uint32_t nitems,
                                   hipStream_t s)
{
    if (nitems == 0)
        return hipSuccess;
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_wide_split_L_batch<LL>(args, items, nitems, s);
        MUCA_WIDE_SPLIT_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_split_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items, uint32_t nitems,
                              hipStream_t s)
{
    if (nitems == 0)
        return hipSuccess;
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_split_L_batch_L<LL>(args, items, nitems, s);
        MUCA_SPLIT_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace muca
