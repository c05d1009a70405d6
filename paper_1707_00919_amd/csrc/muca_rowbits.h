// muca_rowbits.h -- per-lane bit bookkeeping of one walker's current row, shared
// by the fast and split sweep kernels (bit-packed lattice, typewriter order).
//
// For the row being swept a lane keeps
//   up, cur, dn  rows y-1 (already updated this sweep), y (as the row started),
//                y+1 (not yet updated);
//   nb           bit i = 1 iff sites i and i+1 of the row differ (cyclic); it
//                is kept current while the row is swept: flipping site x
//                toggles bits x-1 and x;
//   vi           per site a 2-bit two's-complement field holding
//                (site differs from the site above) + (differs from the site
//                below) - 2, interleaved so that one signed bit-field extract
//                reads it;
//   nb0, f0      nb at the row start and whether site 0 flipped, from which
//                the row's flipped sites are recovered at the row end.
// The number m of neighbours anti-aligned with site x is then
//   m - 2 = popcount(nb & (bits x-1, x)) + vi(x),
// and m - 2 is minus the change of the energy bin if site x flips
// (Delta E = 8 - 4m for the 2D Ising model, Sec. 3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muca {

template <int L>
struct RowBits {
    static constexpr int WPR = (L + 31) / 32;          // 32-bit words per row
    static constexpr int LAST = L - 32 * (WPR - 1);    // sites in the last word
    static constexpr int VIW = (L + 15) / 16;          // words of vi (16 sites each)
    uint32_t up[WPR], cur[WPR], dn[WPR];
    uint32_t nb[WPR], nb0[WPR];
    uint32_t vi[VIW];
    uint32_t f0;
};

// bits 0..15 of x spread to the even bits of the result
__device__ __forceinline__ uint32_t spread16(uint32_t x)
{
    x &= 0xffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

template <int L>
__device__ __forceinline__ void rowbits_begin(RowBits<L>& rb)
{
    using R = RowBits<L>;
#pragma unroll
    for (int w = 0; w < R::WPR; ++w) {
        const uint32_t u = rb.cur[w] ^ rb.up[w];
        const uint32_t d = rb.cur[w] ^ rb.dn[w];
        const uint32_t lo = u ^ d;     // low bit of (u + d - 2)
        const uint32_t hi = ~(u & d);  // high (sign) bit of (u + d - 2)
        if (2 * w < R::VIW)
            rb.vi[2 * w] = spread16(lo) | (spread16(hi) << 1);
        if (2 * w + 1 < R::VIW)
            rb.vi[2 * w + 1] = spread16(lo >> 16) | (spread16(hi >> 16) << 1);
        uint32_t next;  // bit i = site i+1 of the row (cyclic)
        if (w + 1 < R::WPR)
            next = (rb.cur[w] >> 1) | (rb.cur[w + 1] << 31);
        else
            next = (rb.cur[w] >> 1) | ((rb.cur[0] & 1u) << (R::LAST - 1));
        rb.nb[w] = rb.cur[w] ^ next;
        rb.nb0[w] = rb.nb[w];
    }
}

// Row end: the flipped sites F solve F_i ^ F_{i+1} = (nb0 ^ nb)_i with F_0 = f0.
template <int L>
__device__ __forceinline__ void rowbits_end(RowBits<L>& rb)
{
    using R = RowBits<L>;
    uint32_t carry = 0u - rb.f0;  // all ones if site 0 flipped
#pragma unroll
    for (int w = 0; w < R::WPR; ++w) {
        uint32_t p = rb.nb0[w] ^ rb.nb[w];
        p ^= p << 1;
        p ^= p << 2;
        p ^= p << 4;
        p ^= p << 8;
        p ^= p << 16;  // inclusive prefix xor within the word
        uint32_t flips = (p << 1) ^ carry;
        if (w + 1 == R::WPR && R::LAST < 32)
            flips &= (1u << R::LAST) - 1u;
        carry ^= 0u - (p >> 31);
        rb.cur[w] ^= flips;
    }
}

// (neighbours of site X above/below that differ from it) - 2
template <int L, int X>
__device__ __forceinline__ int vert_minus_two(const RowBits<L>& rb)
{
    constexpr int SH = 2 * (X & 15);
    return (int)(rb.vi[X >> 4] << (30 - SH)) >> 30;
}

// popcount of the bond bits X-1 and X (cyclic) of nb, plus acc
template <int L, int X>
__device__ __forceinline__ int bond_count(const uint32_t (&nb)[RowBits<L>::WPR], int acc)
{
    constexpr int XL = (X + L - 1) % L;
    constexpr int W = X >> 5, B = X & 31, WL = XL >> 5, BL = XL & 31;
    if constexpr (W == WL)
        return __builtin_popcount(nb[W] & ((1u << B) | (1u << BL))) + acc;
    else
        return __builtin_popcount(nb[W] & (1u << B)) + __builtin_popcount(nb[WL] & (1u << BL)) + acc;
}

// nb after flipping site X
template <int L, int X>
__device__ __forceinline__ void bond_flip(uint32_t (&nb)[RowBits<L>::WPR])
{
    constexpr int XL = (X + L - 1) % L;
    constexpr int W = X >> 5, B = X & 31, WL = XL >> 5, BL = XL & 31;
    if constexpr (W == WL) {
        nb[W] ^= (1u << B) | (1u << BL);
    } else {
        nb[W] ^= 1u << B;
        nb[WL] ^= 1u << BL;
    }
}

}  // namespace muca
