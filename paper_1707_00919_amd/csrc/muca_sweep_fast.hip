// muca_sweep_fast.hip -- the multicanonical Metropolis sweep with one wave per
// 64 walkers, for lattices whose per-bin state fits in LDS (L <= 64), gfx950.
//
// Same chain as the generic sweep (Sec. 2.3: one lane per walker, all lanes on
// the same site in typewriter order, Philox draws labelled by walker and site,
// acceptance min(1, exp[omega(E') - omega(E)]) as an integer threshold), with
// the per-attempt work cut to what the method needs:
//
//  * Site words (muca_rowbits.h): per group of eight sites one word of the
//    row's bonds and vertical mismatches, so that a site's count of
//    anti-aligned neighbours is one masked popcount; the row's flips are
//    collected as a word and applied at the row's end.
//  * One 28-byte LDS record per energy bin and a chain step that loads both
//    thresholds the next attempt can need while the current one is decided
//    (muca_chain.h).
//  * Thresholds are stored as S = T - 1 in 32 bits and an attempt is accepted
//    iff r <= S, which equals r < T for every T in [1, 2^32].  The host uses
//    this kernel only when no reachable threshold is 0 (then r < T can never
//    hold); otherwise it runs the generic kernel with 64-bit thresholds.
//  * Philox4x32-10 is computed in the chain wave itself, one block of four
//    sites ahead.  (The two-wave split kernel moves it to a second wave; it
//    wins while the device has room for that wave.)
//  * Where the record table is too large for four workgroups per CU (L >= 40)
//    a workgroup holds two or four waves that share one table.
#include "muca_device.h"

#include "muca_chain.h"
#include "philox.h"

namespace muca {
namespace {

// The chain of walker w (one lane) over all sweeps of the launch.
template <int L>
__device__ __forceinline__ void fast_chain(const FastSweepArgs& a, uint32_t w, uint8_t* lds)
{
    using S = ChainShape<L>;
    uint32_t* const mine = a.spins + w;
    const size_t stride = a.wpad;
    ChainState<L> st;
    const LdsRecords recs{lds};
    chain_load<L, LdsRecords>(st, mine, stride, a.energy[w]);
    chain_prime<L>(st, recs);
    const uint32_t live = w < a.walkers ? 1u : 0u;
    for (uint32_t t = 0; t < a.nsweeps; ++t) {
        const uint64_t sweep = a.sweep0 + t;
        const uint32_t inc = t >= a.therm ? live : 0u;
        for (int y = 0; y < L; y += S::RPS) {
            PhiloxDraws draws{(uint32_t)(y * L) >> 2, (uint32_t)sweep, (uint32_t)(sweep >> 32), a.seed, w, {}};
            Words4 rn = draws.first();
            Words4 rc;
            chain_rows<L, S::RPS>(st, rc, rn, draws, recs, inc, mine, stride, y);
        }
    }
    a.energy[w] = chain_finish<L>(st, recs);
}

// One workgroup: `group` covers the 64-walker blocks group * G .. group * G +
// G - 1, one wave each, all sharing one record table; waves past the
// instance's last block only help fill and drain it.  G is
// fast_waves_per_group(L) for single instances; batched rounds may run other
// G (the batch autotuner's choice), with the same results.
template <int L, int G>
__device__ __forceinline__ void sweep_fast_kernel_body(const FastSweepArgs& a, uint32_t group)
{
    static_assert(ChainShape<L>::REC_BYTES == (int)fast_lds_bytes(L), "LDS size formula");
    __shared__ __attribute__((aligned(16))) uint8_t lds[ChainShape<L>::REC_BYTES];

    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t block = group * (uint32_t)G + threadIdx.x / kWave;
    const uint32_t w = block * kWave + lane;

    chain_records_fill<L>(lds, a.table, threadIdx.x, G * kWave);
    __syncthreads();
    if (w < a.wpad)
        fast_chain<L>(a, w, lds);
    __syncthreads();
    chain_records_flush<L>(lds, a.hist, threadIdx.x, G * kWave);
}

template <int L>
__global__ __launch_bounds__(64 * fast_waves_per_group(L)) void sweep_fast_kernel(FastSweepArgs a)
{
    sweep_fast_kernel_body<L, (int)fast_waves_per_group(L)>(a, blockIdx.x);
}

template <int L, int G>
__global__ __launch_bounds__(64 * G) void sweep_fast_kernel_batch(const FastSweepArgs* args, const BatchItem* items)
{
    const BatchItem it = items[blockIdx.x];
    sweep_fast_kernel_body<L, G>(member_args(args, it.member), it.block);
}

template <int L>
hipError_t launch_fast_L_batch_L(uint32_t G, const FastSweepArgs* args, const BatchItem* items, uint32_t n,
                                 hipStream_t s)
{
    switch (G) {
    case 1:
        hipLaunchKernelGGL((sweep_fast_kernel_batch<L, 1>), dim3(n), dim3(kWave), 0, s, args, items);
        break;
    case 2:
        hipLaunchKernelGGL((sweep_fast_kernel_batch<L, 2>), dim3(n), dim3(2 * kWave), 0, s, args, items);
        break;
    case 4:
        hipLaunchKernelGGL((sweep_fast_kernel_batch<L, 4>), dim3(n), dim3(4 * kWave), 0, s, args, items);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L>
hipError_t launch_fast_L(const FastSweepArgs& a, hipStream_t s)
{
    constexpr uint32_t G = fast_waves_per_group(L);
    hipLaunchKernelGGL(sweep_fast_kernel<L>, dim3((a.wpad / kWave + G - 1) / G), dim3(kWave * G), 0, s, a);
    return hipGetLastError();
}

}  // namespace

#define MUCA_FAST_L(X)                                                                        \
    X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(26) X(28) X(30) X(32)    \
    X(34) X(36) X(38) X(40) X(42) X(44) X(46) X(48) X(50) X(52) X(54) X(56) X(58) X(60) X(62) \
    X(64)

bool fast_sweep_supported(uint32_t L)
{
    switch (L) {
#define MUCA_CASE(LL) case LL:
        MUCA_FAST_L(MUCA_CASE)
#undef MUCA_CASE
        return true;
    default:
        return false;
    }
}

hipError_t launch_fast_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s)
{
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_fast_L<LL>(a, s);
        MUCA_FAST_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_fast_batch(uint32_t L, uint32_t G, const FastSweepArgs* args, const BatchItem* items,
                             uint32_t nitems, hipStream_t s)
{
    if (nitems == 0)
        return hipSuccess;
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_fast_L_batch_L<LL>(G, args, items, nitems, s);
        MUCA_FAST_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace muca
