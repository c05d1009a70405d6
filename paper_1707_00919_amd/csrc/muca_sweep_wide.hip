// muca_sweep_wide.hip -- the multicanonical sweep for lattices whose per-bin
// threshold table is too large for LDS (L > 64), gfx950.
//
// Same chain step as the L <= 64 kernels (muca_chain.h: both thresholds the
// next attempt can need are loaded while the current attempt is decided, so
// one load latency is hidden per attempt), with the threshold records --
// 32 bytes per energy bin, the five thresholds S = T - 1 by the number m of
// anti-aligned neighbours, from m = 4 down -- read from global memory through the caches (the
// table, 512 KiB at L = 128, stays in L2), and only the 32-bit histogram
// counters in LDS (64 KiB + 4 B at L = 128).  One wave per 64 walkers,
// Philox4x32-10 computed in place.  Used when no reachable threshold is 0
// (otherwise the generic kernel with 64-bit thresholds runs) and when there
// are more workgroups than fit on the device at once, two per CU at most; with
// fewer, the two-wave form of muca_sweep_split.hip (Philox on its own wave)
// runs the same chain faster.
#include "muca_device.h"

#include "muca_chain.h"
#include "philox.h"

namespace muca {
namespace {

template <int L>
__device__ __forceinline__ void sweep_wide_kernel_body(const FastSweepArgs& a, uint32_t block)
{
    using S = ChainShape<L>;
    constexpr int N = S::N;
    __shared__ __attribute__((aligned(16))) uint32_t counters[N + 1];

    const uint32_t lane = threadIdx.x;
    const uint32_t w = block * kWave + lane;
    for (int k = lane; k <= N; k += kWave)
        counters[k] = 0u;
    __syncthreads();

    uint32_t* const mine = a.spins + w;
    const size_t stride = a.wpad;
    const GlobalRecords recs{reinterpret_cast<const uint8_t*>(a.table) + 8, reinterpret_cast<uint8_t*>(counters)};
    ChainState<L> st;
    chain_load<L, GlobalRecords>(st, mine, stride, a.energy[w]);
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
    __syncthreads();
    for (int k = lane; k <= N; k += kWave) {
        const uint32_t v = counters[k];
        if (v)
            atomicAdd(a.hist + k, (unsigned long long)v);
    }
}

template <int L>
__global__ __launch_bounds__(64) void sweep_wide_kernel(FastSweepArgs a)
{
    sweep_wide_kernel_body<L>(a, blockIdx.x);
}

template <int L>
__global__ __launch_bounds__(64) void sweep_wide_kernel_batch(const FastSweepArgs* args, const BatchItem* items)
{
    const BatchItem it = items[blockIdx.x];
    sweep_wide_kernel_body<L>(member_args(args, it.member), it.block);
}

template <int L>
hipError_t launch_wide_L(const FastSweepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_wide_kernel<L>, dim3(a.wpad / kWave), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

template <int L>
hipError_t launch_wide_L_batch(const FastSweepArgs* args, const BatchItem* items, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_wide_kernel_batch<L>, dim3(n), dim3(kWave), 0, s, args, items);
    return hipGetLastError();
}

}  // namespace

#define MUCA_WIDE_L(X) X(80) X(96) X(112) X(128)

bool wide_sweep_supported(uint32_t L)
{
    switch (L) {
#define MUCA_CASE(LL) case LL:
        MUCA_WIDE_L(MUCA_CASE)
#undef MUCA_CASE
        return true;
    default:
        return false;
    }
}

hipError_t launch_wide_sweep(uint32_t L, const FastSweepArgs& a, hipStream_t s)
{
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_wide_L<LL>(a, s);
        MUCA_WIDE_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_wide_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items, uint32_t nitems,
                             hipStream_t s)
{
    if (nitems == 0)
        return hipSuccess;
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_wide_L_batch<LL>(args, items, nitems, s);
        MUCA_WIDE_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace muca
