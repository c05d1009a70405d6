// muca_sweep_split.hip -- the multicanonical sweep with the random numbers and
// the Metropolis chain on two different waves (gfx950, L <= 64).
//
// Each walker's chain is serial: an attempt's threshold depends on the energy
// the previous attempt left behind (Sec. 2.2-2.3).  With 64 walkers per wave
// and a few thousand walkers per GPU, one wave per SIMD is all there is, so the
// chain's latency, not the chip's issue rate, sets the pace.  This kernel
// shortens it in two ways:
//
//  * A workgroup has two waves for the same 64 walkers.  The producer wave
//    runs Philox4x32-10 for the next loop step (one row, or two when L is not
//    a multiple of 4) and writes the words to an LDS ring; the consumer wave
//    runs only the chain, reading four draws with one 16-byte LDS load.  One
//    barrier per loop step hands a ring slot over.
//  * The consumer resolves attempt x while the two thresholds attempt x+1 can
//    need -- site x kept, or site x flipped, which moves the energy bin and
//    the left-neighbour bond of site x+1 -- are already on their way from LDS.
//    After the compare it selects one.  The LDS round trip is then paid once
//    per two attempts on the critical path instead of once per attempt.
//
// Per-bin LDS records are 28 bytes (7 words: the five thresholds S = T - 1 by
// the number m of anti-aligned neighbours, the histogram counter, one pad
// word): an odd word stride spreads the gathers of 64 lanes over all banks.
// The row bookkeeping (bond words, vertical fields) is in muca_rowbits.h.
#include "muca_device.h"

#include <utility>

#include "muca_rowbits.h"
#include "philox.h"

namespace muca {
namespace {

template <int L>
struct SplitShape {
    static constexpr int N = L * L;
    static constexpr int WPR = (L + 31) / 32;
    static constexpr int LAST = L - 32 * (WPR - 1);
    static constexpr int RPS = (L % 4 == 0) ? 1 : 2;  // rows per loop step
    static constexpr int STEPS = L / RPS;             // loop steps per sweep
    static constexpr int BLOCKS = RPS * L / 4;        // Philox blocks per loop step
    static constexpr int REC = 28;                    // bytes per energy bin
    static constexpr int REC_BYTES = REC * (N + 1);
    static constexpr int SLOT_BYTES = BLOCKS * kWave * 16;
    static constexpr int LDS_BYTES = REC_BYTES + 2 * SLOT_BYTES;
};

template <int L>
struct ChainState {
    RowBits<L> rb;
    uint32_t z;          // byte address of the record of the current bin + 8
    int ms;              // (anti-aligned neighbours of the next site) - 2
    uint32_t thr_keep;   // threshold S of the next site if the previous site
    uint32_t thr_flip;   // was kept / flipped (loads may still be in flight)
    bool prev_flip;      // the previous site flipped
    uint32_t inc_last;   // record flag of the attempt that left the walker in z
};

__device__ __forceinline__ uint32_t lds_u32(const uint8_t* lds, uint32_t byte)
{
    return *reinterpret_cast<const uint32_t*>(lds + byte);
}

template <int L>
__device__ __forceinline__ void chain_row_begin(ChainState<L>& st, const uint8_t* lds)
{
    rowbits_begin<L>(st.rb);
    st.ms = bond_count<L, 0>(st.rb.nb, vert_minus_two<L, 0>(st.rb));
    st.thr_keep = lds_u32(lds, st.z + (uint32_t)(st.ms * 4));
    st.thr_flip = st.thr_keep;
    st.prev_flip = false;
}

// Attempt at site X = P % L; P counts the sites of the loop step.
//
// Order inside one attempt: first the two threshold loads that site X+1 may
// need (they depend only on the state after site X-1), then the threshold of
// site X is picked from the pair loaded one attempt earlier, compared, and the
// state updated.  The scheduling barrier keeps the compiler from moving that
// pick, and the wait on LDS it implies, above the new loads: each load then has
// a whole attempt of independent work to hide behind.
template <int L, int P>
__device__ __forceinline__ void chain_attempt(ChainState<L>& st, Words4& rc, Words4& rn,
                                              uint8_t* lds, uint32_t slot, uint32_t lane,
                                              uint32_t inc)
{
    using S = SplitShape<L>;
    constexpr int X = P % L;
    if constexpr ((P & 3) == 0) {
        rc = rn;
        if constexpr ((P >> 2) + 1 < S::BLOCKS) {
            const uint4 v = *reinterpret_cast<const uint4*>(
                lds + slot + (uint32_t)(((P >> 2) + 1) * kWave + lane) * 16u);
            rn = Words4{{v.x, v.y, v.z, v.w}};
        }
    }
    const uint32_t r = rc.w[P & 3];
    uint32_t nbf[S::WPR];
#pragma unroll
    for (int w = 0; w < S::WPR; ++w)
        nbf[w] = st.rb.nb[w];
    bond_flip<L, X>(nbf);
    const uint32_t zf = st.z - (uint32_t)(st.ms * 28);
    int ms_keep = 0, ms_flip = 0;
    uint32_t next_keep = 0u, next_flip = 0u;
    if constexpr (X + 1 < L) {
        // both possible thresholds of site X+1
        const int v1 = vert_minus_two<L, X + 1>(st.rb);
        ms_keep = bond_count<L, X + 1>(st.rb.nb, v1);
        ms_flip = bond_count<L, X + 1>(nbf, v1);
        next_keep = lds_u32(lds, st.z + (uint32_t)(ms_keep * 4));
        next_flip = lds_u32(lds, zf + (uint32_t)(ms_flip * 4));
    }
    // the bin the previous attempt left the walker in is counted here, after
    // the loads above: LDS answers a wave in order, so the loads do not wait
    // behind this read-modify-write
    atomicAdd(reinterpret_cast<uint32_t*>(lds + st.z + 12), X == 0 ? st.inc_last : inc);
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t thr = st.prev_flip ? st.thr_flip : st.thr_keep;
    const bool accept = r <= thr;
    st.z = accept ? zf : st.z;
#pragma unroll
    for (int w = 0; w < S::WPR; ++w)
        st.rb.nb[w] = accept ? nbf[w] : st.rb.nb[w];
    if constexpr (X == 0)
        st.rb.f0 = accept ? 1u : 0u;
    if constexpr (X + 1 == L)
        st.inc_last = inc;
    if constexpr (X + 1 < L) {
        st.ms = accept ? ms_flip : ms_keep;
        st.thr_keep = next_keep;
        st.thr_flip = next_flip;
        st.prev_flip = accept;
    }
}

template <int L, int RR, int... Xs>
__device__ __forceinline__ void chain_row_sites(ChainState<L>& st, Words4& rc, Words4& rn,
                                                uint8_t* lds, uint32_t slot, uint32_t lane,
                                                uint32_t inc, std::integer_sequence<int, Xs...>)
{
    (chain_attempt<L, RR * L + Xs>(st, rc, rn, lds, slot, lane, inc), ...);
}

template <int L, int RR>
__device__ __forceinline__ void chain_row(ChainState<L>& st, Words4& rc, Words4& rn,
                                          uint8_t* lds, uint32_t slot, uint32_t lane,
                                          uint32_t inc, uint32_t* mine, size_t stride, int y)
{
    constexpr int WPR = SplitShape<L>::WPR;
    const int yy = y + RR;
    const int ynext = (yy + 2) % L;
    uint32_t nx[WPR];
#pragma unroll
    for (int j = 0; j < WPR; ++j)
        nx[j] = mine[(size_t)(ynext * WPR + j) * stride];
    chain_row_begin<L>(st, lds);
    chain_row_sites<L, RR>(st, rc, rn, lds, slot, lane, inc, std::make_integer_sequence<int, L>{});
    rowbits_end<L>(st.rb);
#pragma unroll
    for (int j = 0; j < WPR; ++j) {
        mine[(size_t)(yy * WPR + j) * stride] = st.rb.cur[j];
        st.rb.up[j] = st.rb.cur[j];
        st.rb.cur[j] = st.rb.dn[j];
        st.rb.dn[j] = nx[j];
    }
}

// Producer: the Philox words of every site of loop step s into ring slot s & 1.
template <int L>
__device__ __forceinline__ void produce_step(uint8_t* lds, uint32_t s, const FastSweepArgs& a,
                                             uint32_t walker, uint32_t lane)
{
    using S = SplitShape<L>;
    const uint32_t t = s / S::STEPS;
    const uint32_t y = (s - t * S::STEPS) * S::RPS;
    const uint64_t sweep = a.sweep0 + t;
    const uint32_t blk0 = (y * L) >> 2;
    uint8_t* slot = lds + S::REC_BYTES + (s & 1u) * S::SLOT_BYTES;
#pragma unroll 2
    for (int b = 0; b < S::BLOCKS; ++b) {
        const Words4 r = philox10(blk0 + (uint32_t)b, (uint32_t)sweep, (uint32_t)(sweep >> 32), 0u,
                                  a.seed, walker);
        *reinterpret_cast<uint4*>(slot + (uint32_t)(b * kWave + lane) * 16u) =
            uint4{r.w[0], r.w[1], r.w[2], r.w[3]};
    }
}

template <int L>
__device__ __forceinline__ void sweep_split_kernel_body(const FastSweepArgs& a, uint32_t block)
{
    using S = SplitShape<L>;
    static_assert(S::LDS_BYTES <= 160 * 1024, "records and ring must fit in LDS");
    static_assert(S::LDS_BYTES == (int)split_lds_bytes(L), "LDS size formula");
    constexpr int N = S::N;
    constexpr int WPR = S::WPR;
    __shared__ __attribute__((aligned(16))) uint8_t lds[S::LDS_BYTES];

    const uint32_t lane = threadIdx.x & (kWave - 1);
    const bool consumer = threadIdx.x < kWave;  // wave 0: chain; wave 1: random numbers
    const uint32_t w = block * kWave + lane;
    const uint32_t steps = a.nsweeps * (uint32_t)S::STEPS;

    uint32_t* rec = reinterpret_cast<uint32_t*>(lds);
    for (int i = threadIdx.x; i < 7 * (N + 1); i += 2 * kWave) {
        const int k = i / 7, j = i - 7 * (i / 7);
        rec[i] = j < 5 ? a.table[k * 5 + j] : 0u;
    }
    if (!consumer && steps > 0)
        produce_step<L>(lds, 0u, a, w, lane);
    __syncthreads();

    uint32_t* const mine = a.spins + w;
    const size_t stride = a.wpad;
    ChainState<L> st;
    const uint32_t live = w < a.walkers ? 1u : 0u;
    if (consumer) {
#pragma unroll
        for (int j = 0; j < WPR; ++j) {
            st.rb.up[j] = mine[(size_t)((L - 1) * WPR + j) * stride];
            st.rb.cur[j] = mine[(size_t)j * stride];
            st.rb.dn[j] = mine[(size_t)(WPR + j) * stride];
        }
        st.rb.f0 = 0u;
        st.z = 28u * (uint32_t)((a.energy[w] + 2 * N) >> 2) + 8u;
        st.inc_last = 0u;  // no attempt yet
    }

    for (uint32_t s = 0; s < steps; ++s) {
        if (consumer) {
            const uint32_t t = s / S::STEPS;
            const int y = (int)(s - t * S::STEPS) * S::RPS;
            const uint32_t inc = t >= a.therm ? live : 0u;
            const uint32_t slot = S::REC_BYTES + (s & 1u) * S::SLOT_BYTES;
            const uint4 v = *reinterpret_cast<const uint4*>(lds + slot + lane * 16u);
            Words4 rn = Words4{{v.x, v.y, v.z, v.w}};
            Words4 rc;
            chain_row<L, 0>(st, rc, rn, lds, slot, lane, inc, mine, stride, y);
            if constexpr (S::RPS == 2)
                chain_row<L, 1>(st, rc, rn, lds, slot, lane, inc, mine, stride, y);
        } else if (s + 1 < steps) {
            produce_step<L>(lds, s + 1, a, w, lane);
        }
        __syncthreads();
    }
    if (consumer) {
        atomicAdd(reinterpret_cast<uint32_t*>(lds + st.z + 12), st.inc_last);  // the last attempt
        a.energy[w] = 4 * (int)((st.z - 8u) / 28u) - 2 * N;
    }

    __syncthreads();
    for (int k = threadIdx.x; k <= N; k += 2 * kWave) {
        const uint32_t v = rec[7 * k + 5];
        if (v)
            atomicAdd(a.hist + k, (unsigned long long)v);
    }
}

template <int L>
__global__ __launch_bounds__(128) void sweep_split_kernel(FastSweepArgs a)
{
    sweep_split_kernel_body<L>(a, blockIdx.x);
}

template <int L>
__global__ __launch_bounds__(128) void sweep_split_kernel_batch(const FastSweepArgs* args, const BatchItem* items)
{
    const BatchItem it = items[blockIdx.x];
    sweep_split_kernel_body<L>(args[it.member], it.block);
}

template <int L>
hipError_t launch_split_L_batch_L(const FastSweepArgs* args, const BatchItem* items, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_split_kernel_batch<L>, dim3(n), dim3(2 * kWave), 0, s, args, items);
    return hipGetLastError();
}

template <int L>
hipError_t launch_split_L(const FastSweepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_split_kernel<L>, dim3(a.wpad / kWave), dim3(2 * kWave), 0, s, a);
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
