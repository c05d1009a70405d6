// muca_sweep_fast.hip -- the multicanonical Metropolis sweep for lattices whose
// whole per-bin state fits in LDS (L <= 64), tuned for gfx950.
//
// Same chain as the generic sweep (Sec. 2.3: one lane per walker, all lanes on
// the same site in typewriter order, Philox draws labelled by walker and site,
// acceptance min(1, exp[omega(E') - omega(E)]) as an integer threshold), with
// the per-attempt work cut to what the method needs:
//
//  * Bond words (muca_rowbits.h).  At the start of a row the lane forms a
//    word nb whose bit i says whether sites i and i+1 of the row differ, kept
//    current as spins flip, and per site the count of differing neighbours
//    above and below as a signed 2-bit field; the number m of anti-aligned
//    neighbours of a site is then one popcount and one bit-field extract.
//    The row's flipped sites are recovered from the change of nb at the end.
//  * One LDS record of 28 bytes per energy bin k: the five thresholds of the
//    moves out of k, ordered by m, the bin's histogram counter and a pad word
//    (an odd word stride spreads the gathers of a wave over all LDS banks).
//    A walker keeps a single byte address z = 28k + 8: the threshold of a
//    move with m anti-aligned neighbours sits at z + 4(m - 2), the record of
//    the target bin k' = k + 2 - m at z - 28(m - 2), and the counter at
//    z + 12.
//  * Thresholds are stored as S = T - 1 in 32 bits and an attempt is accepted
//    iff r <= S, which equals r < T for every T in [1, 2^32].  The host uses
//    this kernel only when no reachable threshold is 0 (then r < T can never
//    hold); otherwise it runs the generic kernel with 64-bit thresholds.
//  * The Philox block of the next four sites is computed while the current
//    four attempts wait on LDS.
//  * Where the record table is too large for four workgroups per CU (L >= 40)
//    a workgroup holds two or four waves that share one table.
#include "muca_device.h"

#include <utility>

#include "muca_rowbits.h"
#include "philox.h"

namespace muca {
namespace {

template <int L>
struct FastShape {
    static constexpr int N = L * L;
    static constexpr int WPR = (L + 31) / 32;
    static constexpr int LAST = L - 32 * (WPR - 1);  // sites in the last word of a row
    static constexpr int RPS = (L % 4 == 0) ? 1 : 2;  // rows per loop step: whole Philox blocks
    static constexpr int BLOCKS = RPS * L / 4;        // Philox blocks per loop step
    static constexpr int REC = 28;                    // LDS bytes per energy bin
    static constexpr int LDS_BYTES = REC * (N + 1);
};

struct FastCtx {
    uint32_t blk0;   // Philox block of the first site of the loop step
    uint32_t c1, c2; // sweep counter words
    uint32_t seed, walker;
    uint32_t inc;    // 1 if this sweep is recorded and the walker is live
};

__device__ __forceinline__ uint32_t lds_load(const uint8_t* lds, uint32_t byte)
{
    return *reinterpret_cast<const uint32_t*>(lds + byte);
}

template <int L, int P>
__device__ __forceinline__ void fast_attempt(RowBits<L>& rb, uint32_t& z, uint32_t& inc_last, Words4& rcur,
                                             Words4& rnext, const FastCtx& c, uint8_t* lds)
{
    using S = FastShape<L>;
    constexpr int X = P % L;
    if constexpr ((P & 3) == 0) {
        rcur = rnext;
        if constexpr ((P >> 2) + 1 < S::BLOCKS)
            rnext = philox10(c.blk0 + (uint32_t)((P >> 2) + 1), c.c1, c.c2, 0u, c.seed, c.walker);
    }
    const uint32_t r = rcur.w[P & 3];
    // ms = (anti-aligned neighbours) - 2 = -(change of the energy bin)
    const int ms = bond_count<L, X>(rb.nb, vert_minus_two<L, X>(rb));
    const uint32_t thr = lds_load(lds, z + (uint32_t)(ms * 4));
    // the bin the previous attempt left the walker in, counted after the load
    // so that the load does not wait behind this read-modify-write
    atomicAdd(reinterpret_cast<uint32_t*>(lds + z + 12), X == 0 ? inc_last : c.inc);
    const uint32_t target = z - (uint32_t)(ms * 28);
    const bool accept = r <= thr;
    z = accept ? target : z;
    uint32_t nbf[S::WPR];
#pragma unroll
    for (int w = 0; w < S::WPR; ++w)
        nbf[w] = rb.nb[w];
    bond_flip<L, X>(nbf);
#pragma unroll
    for (int w = 0; w < S::WPR; ++w)
        rb.nb[w] = accept ? nbf[w] : rb.nb[w];
    if constexpr (X == 0)
        rb.f0 = accept ? 1u : 0u;
    if constexpr (X + 1 == L)
        inc_last = c.inc;
}

template <int L, int RR, int... Xs>
__device__ __forceinline__ void fast_row_sites(RowBits<L>& st, uint32_t& z, uint32_t& inc_last, Words4& rcur,
                                               Words4& rnext, const FastCtx& c, uint8_t* lds,
                                               std::integer_sequence<int, Xs...>)
{
    (fast_attempt<L, RR * L + Xs>(st, z, inc_last, rcur, rnext, c, lds), ...);
}

template <int L, int RR>
__device__ __forceinline__ void fast_row_step(RowBits<L>& st, uint32_t& z, uint32_t& inc_last, Words4& rcur,
                                              Words4& rnext, const FastCtx& c, uint8_t* lds,
                                              uint32_t* mine, size_t stride, int y)
{
    constexpr int WPR = FastShape<L>::WPR;
    const int yy = y + RR;
    const int ynext = (yy + 2) % L;
    uint32_t nx[WPR];
#pragma unroll
    for (int j = 0; j < WPR; ++j)
        nx[j] = mine[(size_t)(ynext * WPR + j) * stride];
    rowbits_begin<L>(st);
    fast_row_sites<L, RR>(st, z, inc_last, rcur, rnext, c, lds, std::make_integer_sequence<int, L>{});
    rowbits_end<L>(st);
#pragma unroll
    for (int j = 0; j < WPR; ++j) {
        mine[(size_t)(yy * WPR + j) * stride] = st.cur[j];
        st.up[j] = st.cur[j];
        st.cur[j] = st.dn[j];
        st.dn[j] = nx[j];
    }
}

// The chain of walker w (one lane) over all sweeps of the launch.
template <int L>
__device__ __forceinline__ void fast_chain(const FastSweepArgs& a, uint32_t w, uint8_t* lds)
{
    using S = FastShape<L>;
    constexpr int N = S::N;
    constexpr int WPR = S::WPR;
    uint32_t* const mine = a.spins + w;
    const size_t stride = a.wpad;
    RowBits<L> st;
#pragma unroll
    for (int j = 0; j < WPR; ++j) {
        st.up[j] = mine[(size_t)((L - 1) * WPR + j) * stride];
        st.cur[j] = mine[(size_t)j * stride];
        st.dn[j] = mine[(size_t)(WPR + j) * stride];
    }
    st.f0 = 0u;
    const int k0 = (a.energy[w] + 2 * N) >> 2;
    uint32_t z = 28u * (uint32_t)k0 + 8u;
    uint32_t inc_last = 0u;  // no attempt yet
    const uint32_t live = w < a.walkers ? 1u : 0u;

    FastCtx c;
    c.seed = a.seed;
    c.walker = w;
    for (uint32_t t = 0; t < a.nsweeps; ++t) {
        const uint64_t sweep = a.sweep0 + t;
        c.c1 = (uint32_t)sweep;
        c.c2 = (uint32_t)(sweep >> 32);
        c.inc = t >= a.therm ? live : 0u;
        for (int y = 0; y < L; y += S::RPS) {
            c.blk0 = (uint32_t)(y * L) >> 2;
            Words4 rcur;
            Words4 rnext = philox10(c.blk0, c.c1, c.c2, 0u, c.seed, c.walker);
            fast_row_step<L, 0>(st, z, inc_last, rcur, rnext, c, lds, mine, stride, y);
            if constexpr (S::RPS == 2)
                fast_row_step<L, 1>(st, z, inc_last, rcur, rnext, c, lds, mine, stride, y);
        }
    }
    atomicAdd(reinterpret_cast<uint32_t*>(lds + z + 12), inc_last);  // the last attempt
    a.energy[w] = 4 * (int)((z - 8u) / 28u) - 2 * N;
}

// One workgroup: `group` covers the 64-walker blocks group * G .. group * G +
// G - 1 (G = fast_waves_per_group(L)), one wave each, all sharing one record
// table; waves past the instance's last block only help fill and drain it.
template <int L>
__device__ __forceinline__ void sweep_fast_kernel_body(const FastSweepArgs& a, uint32_t group)
{
    using S = FastShape<L>;
    constexpr int N = S::N;
    constexpr int G = (int)fast_waves_per_group(L);
    static_assert(S::LDS_BYTES == (int)fast_lds_bytes(L), "LDS size formula");
    __shared__ __attribute__((aligned(16))) uint8_t lds[S::LDS_BYTES];

    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t block = group * (uint32_t)G + threadIdx.x / kWave;
    const uint32_t w = block * kWave + lane;

    // records: five thresholds S = T - 1 (by m), a zeroed histogram counter, pad
    uint32_t* rec = reinterpret_cast<uint32_t*>(lds);
    for (int i = threadIdx.x; i < 7 * (N + 1); i += G * kWave) {
        const int k = i / 7, j = i - 7 * (i / 7);
        rec[i] = j < 5 ? a.table[k * 5 + j] : 0u;
    }
    __syncthreads();
    if (w < a.wpad)
        fast_chain<L>(a, w, lds);
    __syncthreads();
    for (int k = threadIdx.x; k <= N; k += G * kWave) {
        const uint32_t v = rec[7 * k + 5];
        if (v)
            atomicAdd(a.hist + k, (unsigned long long)v);
    }
}

template <int L>
__global__ __launch_bounds__(64 * fast_waves_per_group(L)) void sweep_fast_kernel(FastSweepArgs a)
{
    sweep_fast_kernel_body<L>(a, blockIdx.x);
}

template <int L>
__global__ __launch_bounds__(64 * fast_waves_per_group(L)) void sweep_fast_kernel_batch(const FastSweepArgs* args,
                                                                                       const BatchItem* items)
{
    const BatchItem it = items[blockIdx.x];
    sweep_fast_kernel_body<L>(args[it.member], it.block);
}

template <int L>
hipError_t launch_fast_L_batch_L(const FastSweepArgs* args, const BatchItem* items, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_fast_kernel_batch<L>, dim3(n), dim3(kWave * fast_waves_per_group(L)), 0, s, args,
                       items);
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

hipError_t launch_fast_batch(uint32_t L, const FastSweepArgs* args, const BatchItem* items, uint32_t nitems,
                             hipStream_t s)
{
    if (nitems == 0)
        return hipSuccess;
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_fast_L_batch_L<LL>(args, items, nitems, s);
        MUCA_FAST_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace muca
