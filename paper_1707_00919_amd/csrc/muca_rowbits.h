// muca_rowbits.h -- per-lane bookkeeping of one walker's current row, shared by
// the sweep kernels' chain (bit-packed lattice, typewriter order, Sec. 2.3).
//
// A lane keeps the rows y-1 (already updated in this sweep), y (as the row
// started) and y+1 (not yet updated), each as ceil(L/32) words (bit x%32 of
// word x/32 is site x; set = spin +1).  At the row start it forms, for every
// group of eight sites 8i..8i+7, one word R[i] holding all that the eight
// sites' neighbour counts need:
//   bits 0..8    the bonds 8i-1 .. 8i+7 of the row (bond b: sites b and b+1
//                differ; cyclic, bond -1 is bond L-1),
//   bits 16..23  site differs from the site above, for sites 8i..8i+7,
//   bits 24..31  site differs from the site below.
// The number m of neighbours anti-aligned with site x = 8i + j is then the
// popcount of bits j, j+1, 16+j, 24+j of R[i]; the chain carries d = 2 - m,
// the change of the energy bin if site x flips (Delta E = 8 - 4m for the 2D
// Ising model, Sec. 3), which is the popcount of the same bits of ~R[i],
// minus 2.  Flipping site x toggles bond x, the left bond of site x+1 (bit
// j+1 of its word); the last site's right bond is bond L-1, toggled when site
// 0 flips.  The row's flips are collected as words (bit x: site x flipped)
// and applied at the row end.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muca {

template <int L>
struct RowWords {
    static constexpr int WPR = (L + 31) / 32;        // 32-bit words per row
    static constexpr int LAST = L - 32 * (WPR - 1);  // sites in the last word
    static constexpr int RW = (L + 7) / 8;           // site words per row
    uint32_t up[WPR], cur[WPR], dn[WPR];             // rows y-1 (updated), y, y+1
    uint32_t nx[WPR];                                // row y+2
    uint32_t R[RW];
    uint32_t R0next;                                 // R[0] of row y+1 (rows of >= 16 sites)
    uint32_t flips[WPR];
};

// Bond bit x of a row (sites x and x+1, cyclic, differ), word w.
template <int L>
__device__ __forceinline__ uint32_t row_bonds(const uint32_t (&row)[RowWords<L>::WPR], int w)
{
    using R = RowWords<L>;
    uint32_t next;    // bit x = site x+1 of the row (cyclic)
    if constexpr (L == 32)
        next = __builtin_amdgcn_alignbit(row[0], row[0], 1u);
    else if (w + 1 < R::WPR)
        next = __builtin_amdgcn_alignbit(row[w + 1], row[w], 1u);
    else
        next = (row[w] >> 1) | ((row[0] & 1u) << (R::LAST - 1));
    return row[w] ^ next;
}

// Site word 0 (sites 0..7) of a row with the given bond words and rows above
// and below.
template <int L>
__device__ __forceinline__ uint32_t site_word0(const uint32_t (&nb)[RowWords<L>::WPR], uint32_t cur0, uint32_t up0,
                                               uint32_t dn0)
{
    // bond L-1 (the first site's left bond), then bonds 0..7
    const uint32_t last = (nb[RowWords<L>::WPR - 1] >> ((L - 1) & 31)) & 1u;
    const uint32_t bonds = (nb[0] << 1) | last;
    return (bonds & 0x1ffu) | (((cur0 ^ up0) & 0xffu) << 16) | (((cur0 ^ dn0) & 0xffu) << 24);
}

// Site words of the row; word 0 only if with_first.
template <int L>
__device__ __forceinline__ void rowwords_begin(RowWords<L>& rb, bool with_first = true)
{
    using R = RowWords<L>;
    uint32_t nb[R::WPR];  // bond bits: bit x = site x and site x+1 (cyclic) differ
#pragma unroll
    for (int w = 0; w < R::WPR; ++w) {
        nb[w] = row_bonds<L>(rb.cur, w);
        rb.flips[w] = 0u;
    }
    if (with_first)
        rb.R[0] = site_word0<L>(nb, rb.cur[0], rb.up[0], rb.dn[0]);
#pragma unroll
    for (int i = 1; i < R::RW; ++i) {
        // bonds 8i-1 .. 8i+7 (8i-1 is odd, so the shift is never 0), which
        // may straddle two words; bonds past L-1 are never read
        const int b = 8 * i - 1, wb = b >> 5, sh = b & 31;
        const uint32_t hi = (wb + 1 < R::WPR) ? nb[wb + 1] : 0u;
        const uint32_t bonds = __builtin_amdgcn_alignbit(hi, nb[wb], (uint32_t)sh);
        const int w = i >> 2, by = 8 * (i & 3);
        const uint32_t u = ((rb.cur[w] ^ rb.up[w]) >> by) & 0xffu;
        const uint32_t d = ((rb.cur[w] ^ rb.dn[w]) >> by) & 0xffu;
        rb.R[i] = (bonds & 0x1ffu) | (u << 16) | (d << 24);
    }
}

// Site word 0 of the next row, formed while this row is still being swept:
// its sites' upper neighbours are this row's sites 0..7, final once those have
// been visited (flips holds them), and its lower row is the one prefetched.
template <int L>
__device__ __forceinline__ void rowwords_prepare_next(RowWords<L>& rb)
{
    using R = RowWords<L>;
    uint32_t nb[R::WPR];
#pragma unroll
    for (int w = 0; w < R::WPR; ++w)
        nb[w] = row_bonds<L>(rb.dn, w);
    rb.R0next = site_word0<L>(nb, rb.dn[0], rb.cur[0] ^ rb.flips[0], rb.nx[0]);
}

// d = 2 - m of site 8i + J from its site word (m: anti-aligned neighbours),
// with its left bond toggled when flipped_left.
template <int J>
__device__ __forceinline__ int word_d(uint32_t word, bool flipped_left)
{
    constexpr uint32_t MASK = (1u << J) | (1u << (J + 1)) | (1u << (16 + J)) | (1u << (24 + J));
    const uint32_t w = flipped_left ? (word ^ (1u << J)) : word;
    return (int)__builtin_popcount(~w & MASK) - 2;
}

// d = 2 - m of site X, with its left bond toggled when flipped_left (site X-1
// flipped in this row).
template <int L, int X>
__device__ __forceinline__ int site_d(const RowWords<L>& rb, bool flipped_left)
{
    return word_d<X & 7>(rb.R[X >> 3], flipped_left);
}

// After the first site of the row: if it flipped, so did bond L-1, the last
// site's right bond.
template <int L>
__device__ __forceinline__ void rowwords_note_first(RowWords<L>& rb, bool flipped)
{
    constexpr int I = (L - 1) >> 3, J = (L - 1) & 7;
    rb.R[I] = flipped ? (rb.R[I] ^ (1u << (J + 1))) : rb.R[I];
}

// Site X flipped or not.
template <int L, int X>
__device__ __forceinline__ void rowwords_note(RowWords<L>& rb, bool flipped)
{
    rb.flips[X >> 5] |= flipped ? (1u << (X & 31)) : 0u;
}

// Row end: the row as the sweep left it.
template <int L>
__device__ __forceinline__ void rowwords_end(RowWords<L>& rb)
{
#pragma unroll
    for (int w = 0; w < RowWords<L>::WPR; ++w)
        rb.cur[w] ^= rb.flips[w];
}

}  // namespace muca
