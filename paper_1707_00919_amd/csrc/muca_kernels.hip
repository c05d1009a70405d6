// muca_kernels.hip -- gfx950 kernels of libmuca: lattice initialisation and the
// multicanonical Metropolis sweep (Sec. 2.3 of Gross, Zierenberg, Weigel,
// Janke, "Massively parallel multicanonical simulations").
//
// One lane runs one walker (the paper's one thread per walker, Sec. 2.3).  All
// lanes of a wave visit the same site at the same time in typewriter order,
// which is what keeps the lattice accesses of a wave contiguous (the paper's
// synchronous site choice, Sec. 2.3).  Lattices are bit-packed; the three rows
// around the current one live in registers and stream through HBM once per
// row.  The acceptance thresholds and a 32-bit histogram per workgroup live in
// LDS; the histogram is added into the instance's 64-bit histogram with one
// atomic pass at the end of the launch (the paper's single atomically updated
// histogram, Sec. 2.3, with the atomics moved on chip).
#include "muca_device.h"

#include <utility>

#include "philox.h"

namespace muca {
namespace {

template <int L>
struct Shape {
    static constexpr int N = L * L;
    static constexpr int WPR = (L + 31) / 32;
    // rows per step of the row loop: a step always covers whole Philox blocks
    // (4 sites), so the block phase of every site is a compile-time constant.
    static constexpr int RPS = (L % 4 == 0) ? 1 : 2;
    // four uint64 thresholds and one uint32 counter per bin must fit in the
    // 160 KiB of LDS; larger lattices gather thresholds from L2.
    static constexpr bool kTableInLds = 36 * (N + 1) <= 159 * 1024;
};

// Per-lane state of one walker inside the sweep kernel: the rows above, at
// and below the current one (bit-packed) and the current energy bin k.
template <int L>
struct RowWindow {
    uint32_t up[Shape<L>::WPR];
    uint32_t cur[Shape<L>::WPR];
    uint32_t dn[Shape<L>::WPR];
};

struct SweepCtx {
    const uint64_t* table;
    uint32_t* hist;
    uint32_t blk0;  // Philox block of the first site of the loop step
    uint32_t c1, c2;
    uint32_t seed, walker;
    uint32_t inc;   // 1 if this sweep is recorded and the walker is live
};

// One Metropolis attempt at site x = P % L of the current row.  P counts the
// sites of the loop step, so P & 3 is the site's word in its Philox block.
template <int L, int P>
__device__ __forceinline__ void attempt(RowWindow<L>& rw, int& k, Words4& r4, const SweepCtx& c)
{
    constexpr int X = P % L;
    constexpr int XL = (X + L - 1) % L;
    constexpr int XR = (X + 1) % L;
    if constexpr ((P & 3) == 0)
        r4 = philox10(c.blk0 + (uint32_t)(P >> 2), c.c1, c.c2, 0u, c.seed, c.walker);
    const uint32_t r = r4.w[P & 3];
    const uint32_t s = (rw.cur[X >> 5] >> (X & 31)) & 1u;
    const uint32_t sl = (rw.cur[XL >> 5] >> (XL & 31)) & 1u;
    const uint32_t sr = (rw.cur[XR >> 5] >> (XR & 31)) & 1u;
    const uint32_t su = (rw.up[X >> 5] >> (X & 31)) & 1u;
    const uint32_t sd = (rw.dn[X >> 5] >> (X & 31)) & 1u;
    // m = neighbours anti-aligned with s: dE = 8 - 4m, target bin k + 2 - m
    const uint32_t m = (s ^ sl) + (s ^ sr) + (s ^ su) + (s ^ sd);
    const uint32_t slot = m - (m > 2u ? 1u : 0u);
    const uint64_t thr = c.table[k * 4 + (int)slot];
    const bool accept = (m == 2u) || ((uint64_t)r < thr);
    if (accept) {
        rw.cur[X >> 5] ^= 1u << (X & 31);
        k += 2 - (int)m;
    }
    atomicAdd(&c.hist[k], c.inc);
}

template <int L, int RR, int... Xs>
__device__ __forceinline__ void row_sites(RowWindow<L>& rw, int& k, Words4& r4, const SweepCtx& c,
                                          std::integer_sequence<int, Xs...>)
{
    (attempt<L, RR * L + Xs>(rw, k, r4, c), ...);
}

// Row RR of a loop step that starts at row y: prefetch row y+RR+2, run the
// row's L attempts, write the row back and slide the window down by one.
template <int L, int RR>
__device__ __forceinline__ void row_step(RowWindow<L>& rw, int& k, Words4& r4, const SweepCtx& c,
                                         uint32_t* mine, size_t stride, int y)
{
    constexpr int WPR = Shape<L>::WPR;
    const int yy = y + RR;
    const int ynext = (yy + 2) % L;
    uint32_t nx[WPR];
#pragma unroll
    for (int j = 0; j < WPR; ++j)
        nx[j] = mine[(size_t)(ynext * WPR + j) * stride];
    row_sites<L, RR>(rw, k, r4, c, std::make_integer_sequence<int, L>{});
#pragma unroll
    for (int j = 0; j < WPR; ++j) {
        mine[(size_t)(yy * WPR + j) * stride] = rw.cur[j];
        rw.up[j] = rw.cur[j];
        rw.cur[j] = rw.dn[j];
        rw.dn[j] = nx[j];
    }
}

template <int L>
__device__ __forceinline__ void sweep_kernel_body(const SweepArgs& a, uint32_t block)
{
    using S = Shape<L>;
    constexpr int N = S::N;
    constexpr int WPR = S::WPR;
    constexpr int RPS = S::RPS;
    __shared__ uint64_t lds_table[S::kTableInLds ? 4 * (N + 1) : 1];
    __shared__ uint32_t lds_hist[N + 1];

    const uint32_t lane = threadIdx.x;
    const uint32_t w = block * kWave + lane;

    if constexpr (S::kTableInLds) {
        for (int e = lane; e < 4 * (N + 1); e += kWave)
            lds_table[e] = a.table[e];
    }
    for (int b = lane; b <= N; b += kWave)
        lds_hist[b] = 0u;
    __syncthreads();

    uint32_t* const mine = a.spins + w;
    const size_t stride = a.wpad;

    RowWindow<L> rw;
#pragma unroll
    for (int j = 0; j < WPR; ++j) {
        rw.up[j] = mine[(size_t)((L - 1) * WPR + j) * stride];
        rw.cur[j] = mine[(size_t)j * stride];
        rw.dn[j] = mine[(size_t)(WPR + j) * stride];
    }
    int k = (a.energy[w] + 2 * N) >> 2;
    const uint32_t live = w < a.walkers ? 1u : 0u;

    SweepCtx c;
    c.table = S::kTableInLds ? lds_table : a.table;
    c.hist = lds_hist;
    c.seed = a.seed;
    c.walker = w;
    for (uint32_t t = 0; t < a.nsweeps; ++t) {
        const uint64_t sweep = a.sweep0 + t;
        c.c1 = (uint32_t)sweep;
        c.c2 = (uint32_t)(sweep >> 32);
        c.inc = t >= a.therm ? live : 0u;
        for (int y = 0; y < L; y += RPS) {
            c.blk0 = (uint32_t)(y * L) >> 2;
            Words4 r4 = {{0u, 0u, 0u, 0u}};
            row_step<L, 0>(rw, k, r4, c, mine, stride, y);
            if constexpr (RPS == 2)
                row_step<L, 1>(rw, k, r4, c, mine, stride, y);
        }
    }
    a.energy[w] = 4 * k - 2 * N;

    __syncthreads();
    for (int b = lane; b <= N; b += kWave) {
        const uint32_t v = lds_hist[b];
        if (v)
            atomicAdd(a.hist + b, (unsigned long long)v);
    }
}

// Initial spins: +1 iff the top bit of the INIT-domain draw (counter word 3 = 1,
// sweep 0) is set; then the energy from the packed lattice, E = 2u - 2N with u
// the number of unsatisfied bonds.  One lane per walker; runs once.
__global__ __launch_bounds__(256) void init_kernel(InitArgs a)
{
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= a.wpad)
        return;
    const uint32_t L = a.L, N = L * L, wpr = (L + 31u) / 32u;
    uint32_t* const mine = a.spins + w;
    const size_t stride = a.wpad;
    for (uint32_t y = 0; y < L; ++y) {
        for (uint32_t j = 0; j < wpr; ++j) {
            uint32_t word = 0u;
            for (uint32_t b = 0; b < 32u && j * 32u + b < L; ++b) {
                const uint32_t i = y * L + j * 32u + b;
                const Words4 r = philox10(i >> 2, 0u, 0u, 1u, a.seed, w);
                word |= (r.w[i & 3u] >> 31) << b;
            }
            mine[(size_t)(y * wpr + j) * stride] = word;
        }
    }
    uint32_t unsat = 0;
    for (uint32_t y = 0; y < L; ++y) {
        const uint32_t yd = (y + 1u) % L;
        for (uint32_t x = 0; x < L; ++x) {
            const uint32_t xr = (x + 1u) % L;
            const uint32_t s = (mine[(size_t)(y * wpr + x / 32u) * stride] >> (x % 32u)) & 1u;
            const uint32_t r = (mine[(size_t)(y * wpr + xr / 32u) * stride] >> (xr % 32u)) & 1u;
            const uint32_t d = (mine[(size_t)(yd * wpr + x / 32u) * stride] >> (x % 32u)) & 1u;
            unsat += (s ^ r) + (s ^ d);
        }
    }
    a.energy[w] = 2 * (int32_t)unsat - 2 * (int32_t)N;
}

__global__ __launch_bounds__(256) void fill_u64_kernel(unsigned long long* p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0ull;
}

// Part of one sweep: the attempts at sites site_begin .. site_end-1 (site i
// at x = i mod L, y = i div L), for calls that start or stop inside a sweep.
// A plain lane-per-walker loop on the lattice in memory: it runs at most one
// sweep per call, next to whole-sweep launches of the kernels above.
template <bool kFast>
__global__ __launch_bounds__(64) void sweep_range_kernel(RangeArgs a)
{
    extern __shared__ uint32_t range_hist[];
    const uint32_t L = a.L, N = L * L, wpr = (L + 31u) / 32u;
    const uint32_t lane = threadIdx.x;
    const uint32_t w = blockIdx.x * kWave + lane;
    for (uint32_t b = lane; b <= N; b += kWave)
        range_hist[b] = 0u;
    __syncthreads();
    uint32_t* const mine = a.spins + w;
    const size_t stride = a.wpad;
    const uint32_t live = w < a.walkers ? 1u : 0u;
    const uint32_t c1 = (uint32_t)a.sweep, c2 = (uint32_t)(a.sweep >> 32);
    int k = (a.energy[w] + 2 * (int)N) >> 2;
    for (uint32_t i = a.site_begin; i < a.site_end; ++i) {
        const uint32_t x = i % L, y = i / L;
        const uint32_t xl = x == 0 ? L - 1 : x - 1, xr = x + 1 == L ? 0 : x + 1;
        const uint32_t yu = y == 0 ? L - 1 : y - 1, yd = y + 1 == L ? 0 : y + 1;
        uint32_t* const word = mine + (size_t)(y * wpr + x / 32u) * stride;
        const uint32_t cur = *word;
        const uint32_t s = (cur >> (x % 32u)) & 1u;
        const uint32_t sl = (mine[(size_t)(y * wpr + xl / 32u) * stride] >> (xl % 32u)) & 1u;
        const uint32_t sr = (mine[(size_t)(y * wpr + xr / 32u) * stride] >> (xr % 32u)) & 1u;
        const uint32_t su = (mine[(size_t)(yu * wpr + x / 32u) * stride] >> (x % 32u)) & 1u;
        const uint32_t sd = (mine[(size_t)(yd * wpr + x / 32u) * stride] >> (x % 32u)) & 1u;
        const uint32_t m = (s ^ sl) + (s ^ sr) + (s ^ su) + (s ^ sd);
        const uint32_t r = philox10(i >> 2, c1, c2, 0u, a.seed, w).w[i & 3u];
        bool accept;
        if constexpr (kFast) {
            accept = r <= static_cast<const uint32_t*>(a.table)[k * (int)a.table_stride + 4 - (int)m];
        } else {
            const uint32_t slot = m - (m > 2u ? 1u : 0u);
            accept = (m == 2u) || ((uint64_t)r < static_cast<const uint64_t*>(a.table)[k * 4 + (int)slot]);
        }
        if (accept) {
            *word = cur ^ (1u << (x % 32u));
            k += 2 - (int)m;
        }
        if (i >= a.rec_begin)
            atomicAdd(&range_hist[k], live);
    }
    a.energy[w] = 4 * k - 2 * (int)N;
    __syncthreads();
    for (uint32_t b = lane; b <= N; b += kWave) {
        const uint32_t v = range_hist[b];
        if (v)
            atomicAdd(a.hist + b, (unsigned long long)v);
    }
}

template <int L>
__global__ __launch_bounds__(64) void sweep_kernel(SweepArgs a)
{
    sweep_kernel_body<L>(a, blockIdx.x);
}

template <int L>
__global__ __launch_bounds__(64) void sweep_kernel_batch(const SweepArgs* args, const BatchItem* items)
{
    const BatchItem it = items[blockIdx.x];
    sweep_kernel_body<L>(member_args(args, it.member), it.block);
}

template <int L>
hipError_t launch_sweep_L_batch_L(const SweepArgs* args, const BatchItem* items, uint32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_kernel_batch<L>, dim3(n), dim3(kWave), 0, s, args, items);
    return hipGetLastError();
}

template <int L>
hipError_t launch_sweep_L(const SweepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_kernel<L>, dim3(a.wpad / kWave), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

}  // namespace

#define MUCA_FOR_EACH_L(X)                                                                    \
    X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(26) X(28) X(30) X(32)    \
    X(34) X(36) X(38) X(40) X(42) X(44) X(46) X(48) X(50) X(52) X(54) X(56) X(58) X(60) X(62) \
    X(64) X(80) X(96) X(112) X(128)

bool sweep_supported(uint32_t L)
{
    switch (L) {
#define MUCA_CASE(LL) case LL:
        MUCA_FOR_EACH_L(MUCA_CASE)
#undef MUCA_CASE
        return true;
    default:
        return false;
    }
}

hipError_t launch_sweep(uint32_t L, const SweepArgs& a, hipStream_t s)
{
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_sweep_L<LL>(a, s);
        MUCA_FOR_EACH_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_init(const InitArgs& a, hipStream_t s)
{
    const uint32_t threads = 256;
    hipLaunchKernelGGL(init_kernel, dim3((a.wpad + threads - 1) / threads), dim3(threads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, size_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    const uint32_t threads = 256;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + threads - 1) / threads)),
                       dim3(threads), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_sweep_range(const RangeArgs& a, hipStream_t s)
{
    if (a.site_begin >= a.site_end)
        return hipSuccess;
    if (a.L < 4 || a.L > 128 || a.site_end > a.L * a.L || a.wpad % kWave != 0)
        return hipErrorInvalidValue;
    // one 32-bit counter per bin: up to 64 KiB + 4 B at L = 128
    const size_t lds = ((size_t)a.L * a.L + 1) * sizeof(uint32_t);
    constexpr int kMaxLds = 128 * 128 * 4 + 4;
    if (a.table_stride) {
        static const hipError_t attr = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&sweep_range_kernel<true>), hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
        if (attr != hipSuccess)
            return attr;
        hipLaunchKernelGGL(sweep_range_kernel<true>, dim3(a.wpad / kWave), dim3(kWave), lds, s, a);
    } else {
        static const hipError_t attr = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&sweep_range_kernel<false>), hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
        if (attr != hipSuccess)
            return attr;
        hipLaunchKernelGGL(sweep_range_kernel<false>, dim3(a.wpad / kWave), dim3(kWave), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_batch(uint32_t L, const SweepArgs* args, const BatchItem* items, uint32_t nitems,
                              hipStream_t s)
{
    if (nitems == 0)
        return hipSuccess;
    switch (L) {
#define MUCA_CASE(LL) \
    case LL:          \
        return launch_sweep_L_batch_L<LL>(args, items, nitems, s);
        MUCA_FOR_EACH_L(MUCA_CASE)
#undef MUCA_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace muca
