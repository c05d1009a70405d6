// muca_chain.h -- the per-walker Metropolis chain of one row, shared by the
// one-wave (fast), two-wave (split) and wide sweep kernels.
//
// One lane runs one walker; all lanes of a wave are on the same site
// (typewriter order, Sec. 2.3).  The walker's energy bin k is kept as the byte
// address z = 28k + 8 of its 28-byte LDS record (five thresholds S = T - 1
// by the number m of anti-aligned neighbours, from m = 4 down to m = 0, the
// bin's histogram counter, a pad word).  A site is described by d = 2 - m,
// the bin change if it flips: the threshold of its move is at z + 4d, the
// target bin's record at z + 28d, the counter at z + 12.
//
// Each walker's chain is serial (the energy after one attempt picks the next
// threshold), so a chain step's latency sets the pace.  The step hides the
// LDS round trip of the threshold: while attempt x is being decided, the two
// thresholds attempt x+1 can need -- site x kept, or site x flipped (which
// moves the bin and the left-neighbour bond of site x+1) -- are already
// loading; after the compare the step picks one.  The bin an attempt leaves
// the walker in is counted one attempt later, after the next loads are
// issued, since LDS answers a wave's requests in order.  The row bookkeeping
// is in muca_rowbits.h.
//
// Where the records live is a Records policy: LdsRecords (28-byte records in
// LDS, counter inside, L <= 64) or GlobalRecords (32-byte threshold records in
// global memory, read through the caches, with the counters alone in LDS --
// for L > 64, whose tables do not fit in LDS).
//
// The random words come from a Draws source: first() returns the four Philox
// words of block 0 of the current loop step, and advance<B, PART>(rn), called
// at the attempts with P & 3 = PART = 0..3 of the block before B, delivers
// block B into rn by the last of those calls (an LDS ring filled by a producer
// wave does it in one load; Philox computed in place spreads its ten rounds
// over the four attempts, so that they fill the chain's dependency stalls).
#pragma once

#include <utility>

#include "muca_device.h"
#include "muca_rowbits.h"
#include "philox.h"

namespace muca {

template <int L>
struct ChainShape {
    static constexpr int N = L * L;
    static constexpr int WPR = (L + 31) / 32;
    static constexpr int RPS = (L % 4 == 0) ? 1 : 2;  // rows per loop step: whole Philox blocks
    static constexpr int STEPS = L / RPS;             // loop steps per sweep
    static constexpr int BLOCKS = RPS * L / 4;        // Philox blocks per loop step
    static constexpr int REC = 28;                    // LDS bytes per energy bin
    static constexpr int REC_BYTES = REC * (N + 1);
};

// 28-byte records in LDS: z = 28k + 8, threshold of the move with bin
// change d = 2 - m at z + 4d, counter at z + 12.
struct LdsRecords {
    uint8_t* lds;
    __device__ __forceinline__ static uint32_t z_of(int k) { return 28u * (uint32_t)k + 8u; }
    __device__ __forceinline__ static int k_of(uint32_t z) { return (int)((z - 8u) / 28u); }
    // the record of the bin d away
    __device__ __forceinline__ static uint32_t target(uint32_t z, int d) { return z + (uint32_t)(d * 28); }
    __device__ __forceinline__ uint32_t thr(uint32_t z, int d) const
    {
        const uint32_t byte = z + (uint32_t)(d * 4);  // in range: d * 4 >= -8 and z >= 8
        return *reinterpret_cast<const uint32_t*>(lds + byte);
    }
    __device__ __forceinline__ void count(uint32_t z, uint32_t inc) const
    {
        atomicAdd(reinterpret_cast<uint32_t*>(lds + z + 12), inc);
    }
};

// 32-byte threshold records in global memory (S by m at bytes 4(4 - m) of
// record k): z = 32k, threshold of the move with bin change d = 2 - m at
// z + 8 + 4d; the counter of bin k is word k of an LDS array, at byte z / 8.
struct GlobalRecords {
    const uint8_t* table8;  // the table + 8 bytes
    uint8_t* counters;
    __device__ __forceinline__ static uint32_t z_of(int k) { return 32u * (uint32_t)k; }
    __device__ __forceinline__ static int k_of(uint32_t z) { return (int)(z >> 5); }
    // the record of the bin d away
    __device__ __forceinline__ static uint32_t target(uint32_t z, int d) { return z + ((uint32_t)d << 5); }
    __device__ __forceinline__ uint32_t thr(uint32_t z, int d) const
    {
        // z + 4d, formed in 32 bits, is never negative for a move a walker
        // can propose (in bin 0 every site has d = 2; every other reachable
        // bin has z >= 64), so no wrapped term is added to the 64-bit pointer
        const uint32_t byte = z + (uint32_t)(d * 4);
        return *reinterpret_cast<const uint32_t*>(table8 + byte);
    }
    __device__ __forceinline__ void count(uint32_t z, uint32_t inc) const
    {
        atomicAdd(reinterpret_cast<uint32_t*>(counters + (z >> 3)), inc);
    }
};

// The chain's random words computed in place: block B of the loop step that
// starts at Philox block blk0, its ten rounds spread 3 + 3 + 2 + 2 over the
// four attempts before it is needed.
struct PhiloxDraws {
    uint32_t blk0, c1, c2, seed, walker;
    PhiloxState next;
    __device__ __forceinline__ Words4 first() const { return philox10(blk0, c1, c2, 0u, seed, walker); }
    template <int B, int PART>
    __device__ __forceinline__ void advance(Words4& rn)
    {
        if constexpr (PART == 0) {
            next = PhiloxState{blk0 + (uint32_t)B, c1, c2, 0u, seed, walker};
            philox_rounds<0, 3>(next);
        } else if constexpr (PART == 1) {
            philox_rounds<3, 6>(next);
        } else if constexpr (PART == 2) {
            philox_rounds<6, 8>(next);
        } else {
            philox_rounds<8, 10>(next);
            rn = Words4{{next.c0, next.c1, next.c2, next.c3}};
        }
    }
};

template <int L>
struct ChainState {
    RowWords<L> rb;
    uint32_t z;          // the current bin's record address (Records::z_of)
    int d;               // 2 - (anti-aligned neighbours of the next site)
    uint32_t thr_keep;   // threshold S of the next site if the previous site
    uint32_t thr_flip;   // was kept / flipped (loads may still be in flight)
    bool prev_flip;      // the previous site flipped
    uint32_t inc_last;   // record flag of the attempt that left the walker in z
    int d_next_keep;     // d = 2 - m of the site after the next one, if the next
    int d_next_flip;     // site is kept / flips
};

// Fills the records: five thresholds S = T - 1 (by m) from table[k*5 + m], a
// zeroed counter, a pad word.  All threads of the workgroup take part.
template <int L>
__device__ __forceinline__ void chain_records_fill(uint8_t* lds, const uint32_t* table, int first, int stride)
{
    constexpr int N = L * L;
    uint32_t* rec = reinterpret_cast<uint32_t*>(lds);
    for (int i = first; i < 7 * (N + 1); i += stride) {
        const int k = i / 7, j = i - 7 * (i / 7);
        rec[i] = j < 5 ? table[k * 5 + j] : 0u;
    }
}

// Adds the records' counters into the instance histogram (one atomic pass).
template <int L>
__device__ __forceinline__ void chain_records_flush(const uint8_t* lds, unsigned long long* hist, int first,
                                                    int stride)
{
    constexpr int N = L * L;
    const uint32_t* rec = reinterpret_cast<const uint32_t*>(lds);
    for (int k = first; k <= N; k += stride) {
        const uint32_t v = rec[7 * k + 5];
        if (v)
            atomicAdd(hist + k, (unsigned long long)v);
    }
}

// Walker state from its lattice and energy; no attempt counted yet.
template <int L, class R>
__device__ __forceinline__ void chain_load(ChainState<L>& st, const uint32_t* mine, size_t stride, int32_t energy)
{
    constexpr int WPR = ChainShape<L>::WPR;
#pragma unroll
    for (int j = 0; j < WPR; ++j) {
        st.rb.up[j] = mine[(size_t)((L - 1) * WPR + j) * stride];
        st.rb.cur[j] = mine[(size_t)j * stride];
        st.rb.dn[j] = mine[(size_t)(WPR + j) * stride];
    }
    st.z = R::z_of((energy + 2 * L * L) >> 2);
    st.inc_last = 0u;
}

// Counts the bin of the launch's last attempt; returns the walker's energy.
template <int L, class R>
__device__ __forceinline__ int32_t chain_finish(ChainState<L>& st, const R& recs)
{
    recs.count(st.z, st.inc_last);
    return 4 * (int32_t)R::k_of(st.z) - 2 * L * L;
}

// Rows of 16 sites or more run back to back: while row y is swept, the chain
// forms the first site word of row y+1 and, at row y's last attempt, loads the
// two thresholds row y+1's first site can need (row y's last site kept or
// flipped), as for any other site.  Shorter rows start with a load.
template <int L>
struct Seamless {
    static constexpr bool value = L >= 16;
};

// Before the launch's first row: its first site word, the counts of sites 0
// and 1, and site 0's threshold (rows of 16 sites or more).
template <int L, class R>
__device__ __forceinline__ void chain_prime(ChainState<L>& st, const R& recs)
{
    if constexpr (Seamless<L>::value) {
        uint32_t nb[RowWords<L>::WPR];
#pragma unroll
        for (int w = 0; w < RowWords<L>::WPR; ++w)
            nb[w] = row_bonds<L>(st.rb.cur, w);
        st.rb.R0next = site_word0<L>(nb, st.rb.cur[0], st.rb.up[0], st.rb.dn[0]);
        st.d = word_d<0>(st.rb.R0next, false);
        st.d_next_keep = word_d<1>(st.rb.R0next, false);
        st.d_next_flip = word_d<1>(st.rb.R0next, true);
        st.thr_keep = recs.thr(st.z, st.d);
        st.thr_flip = st.thr_keep;
        st.prev_flip = false;
    }
}

template <int L, class R>
__device__ __forceinline__ void chain_row_begin(ChainState<L>& st, const R& recs)
{
    if constexpr (Seamless<L>::value) {
        st.rb.R[0] = st.rb.R0next;
        rowwords_begin<L>(st.rb, false);
    } else {
        rowwords_begin<L>(st.rb);
        st.d = site_d<L, 0>(st.rb, false);
        st.d_next_keep = site_d<L, 1>(st.rb, false);
        st.d_next_flip = site_d<L, 1>(st.rb, true);
        st.thr_keep = recs.thr(st.z, st.d);
        st.thr_flip = st.thr_keep;
        st.prev_flip = false;
    }
}

// Attempt at site X of the row; P counts the sites of the loop step.
//
// Order inside one attempt: first the two threshold loads that site X+1 may
// need (they depend only on the state after site X-1: its left bond, to site
// X, is flipped iff site X flips now) and the inline count of the previous
// attempt's bin; then the threshold of site X is picked from the pair loaded
// one attempt earlier and compared; then the neighbour counts of site X+2 are
// formed, filling the wait the compare's mask needs before the selects that
// read it; then the state is updated.  The scheduling barriers keep the
// compiler from moving the pick, and the wait on LDS it implies, above the
// new loads (each load then has a whole attempt of independent work to hide
// behind), and the counts between the compare and the selects.  For the last
// site, the right bond (to site 0) already carries site 0's flip
// (rowwords_note_first).
template <int L, int X, int P, int BLOCKS, class R, class Draws>
__device__ __forceinline__ void chain_attempt(ChainState<L>& st, Words4& rc, Words4& rn, Draws& draws,
                                              const R& recs, uint32_t inc)
{
    if constexpr ((P & 3) == 0)
        rc = rn;
    if constexpr ((P >> 2) + 1 < BLOCKS)
        draws.template advance<(P >> 2) + 1, (P & 3)>(rn);
    const uint32_t r = rc.w[P & 3];
    const uint32_t zf = R::target(st.z, st.d);
    const int d_keep = st.d_next_keep, d_flip = st.d_next_flip;
    uint32_t next_keep = 0u, next_flip = 0u;
    constexpr bool SEAM = Seamless<L>::value;
    // the next site: X+1 of this row, or (seamless rows) site 0 of the next
    if constexpr (X + 1 < L || SEAM) {
        next_keep = recs.thr(st.z, d_keep);
        next_flip = recs.thr(zf, d_flip);
    }
    recs.count(st.z, X == 0 ? st.inc_last : inc);
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t thr = st.prev_flip ? st.thr_flip : st.thr_keep;
    const bool accept = r <= thr;
    __builtin_amdgcn_sched_barrier(0);
    // the site after the next one; the next row's first sites do not
    // neighbour this row's last one, so only site 1's left bond depends on
    // the branch
    if constexpr (SEAM && X + 3 == L)
        rowwords_prepare_next<L>(st.rb);
    if constexpr (X + 2 < L) {
        st.d_next_keep = site_d<L, X + 2>(st.rb, false);
        st.d_next_flip = site_d<L, X + 2>(st.rb, true);
    } else if constexpr (SEAM && X + 2 == L) {
        st.d_next_keep = word_d<0>(st.rb.R0next, false);
        st.d_next_flip = st.d_next_keep;
    } else if constexpr (SEAM && X + 1 == L) {
        st.d_next_keep = word_d<1>(st.rb.R0next, false);
        st.d_next_flip = word_d<1>(st.rb.R0next, true);
    }
    __builtin_amdgcn_sched_barrier(0);
    st.z = accept ? zf : st.z;
    rowwords_note<L, X>(st.rb, accept);
    if constexpr (X == 0)
        rowwords_note_first<L>(st.rb, accept);
    if constexpr (X + 1 == L)
        st.inc_last = inc;
    if constexpr (X + 1 < L || SEAM) {
        st.d = accept ? d_flip : d_keep;
        st.thr_keep = next_keep;
        st.thr_flip = next_flip;
        st.prev_flip = accept;
    }
}

template <int L, int X0, int P0, int BLOCKS, class R, class Draws, int... Xs>
__device__ __forceinline__ void chain_row_sites(ChainState<L>& st, Words4& rc, Words4& rn, Draws& draws,
                                                const R& recs, uint32_t inc, std::integer_sequence<int, Xs...>)
{
    (chain_attempt<L, X0 + Xs, P0 + Xs, BLOCKS>(st, rc, rn, draws, recs, inc), ...);
}

// Row yy's start: prefetch row yy+2 and form the row's site words.
template <int L, class R>
__device__ __forceinline__ void chain_row_open(ChainState<L>& st, const R& recs, const uint32_t* mine, size_t stride,
                                               uint32_t yy)
{
    constexpr int WPR = ChainShape<L>::WPR;
    const uint32_t ynext = yy + 2u < (uint32_t)L ? yy + 2u : yy + 2u - (uint32_t)L;
#pragma unroll
    for (int j = 0; j < WPR; ++j)
        st.rb.nx[j] = mine[(size_t)(ynext * WPR + j) * stride];
    chain_row_begin<L>(st, recs);
}

// Row yy's end: write the row back and slide the window down by one.
template <int L>
__device__ __forceinline__ void chain_row_close(ChainState<L>& st, uint32_t* mine, size_t stride, uint32_t yy)
{
    constexpr int WPR = ChainShape<L>::WPR;
    rowwords_end<L>(st.rb);
#pragma unroll
    for (int j = 0; j < WPR; ++j) {
        mine[(size_t)(yy * WPR + j) * stride] = st.rb.cur[j];
        st.rb.up[j] = st.rb.cur[j];
        st.rb.cur[j] = st.rb.dn[j];
        st.rb.dn[j] = st.rb.nx[j];
    }
}

// Row RR of a loop step of BLOCKS Philox blocks that starts at row y: its L
// attempts between the row's start and end.
template <int L, int RR, int BLOCKS, class R, class Draws>
__device__ __forceinline__ void chain_row(ChainState<L>& st, Words4& rc, Words4& rn, Draws& draws,
                                          const R& recs, uint32_t inc, uint32_t* mine, size_t stride, int y)
{
    const uint32_t yy = (uint32_t)(y + RR);
    chain_row_open<L>(st, recs, mine, stride, yy);
    chain_row_sites<L, 0, RR * L, BLOCKS>(st, rc, rn, draws, recs, inc, std::make_integer_sequence<int, L>{});
    chain_row_close<L>(st, mine, stride, yy);
}

template <int L, int RPS, class R, class Draws, int... RRs>
__device__ __forceinline__ void chain_rows_seq(ChainState<L>& st, Words4& rc, Words4& rn, Draws& draws, const R& recs,
                                               uint32_t inc, uint32_t* mine, size_t stride, int y,
                                               std::integer_sequence<int, RRs...>)
{
    (chain_row<L, RRs, RPS * L / 4>(st, rc, rn, draws, recs, inc, mine, stride, y), ...);
}

// The RPS rows y .. y+RPS-1 of one loop step; rn holds the step's first
// Philox block.
template <int L, int RPS, class R, class Draws>
__device__ __forceinline__ void chain_rows(ChainState<L>& st, Words4& rc, Words4& rn, Draws& draws, const R& recs,
                                           uint32_t inc, uint32_t* mine, size_t stride, int y)
{
    static_assert((RPS * L) % 4 == 0, "a loop step is whole Philox blocks");
    chain_rows_seq<L, RPS>(st, rc, rn, draws, recs, inc, mine, stride, y, std::make_integer_sequence<int, RPS>{});
}

// Sites X0 .. X0+NX-1 of the current row as one loop step of whole Philox
// blocks (a part of a row between chain_row_open and chain_row_close); rn
// holds the step's first block.
template <int L, int X0, int NX, class R, class Draws>
__device__ __forceinline__ void chain_row_part(ChainState<L>& st, Words4& rc, Words4& rn, Draws& draws,
                                               const R& recs, uint32_t inc)
{
    static_assert(X0 % 4 == 0 && NX % 4 == 0 && X0 + NX <= L, "a loop step is whole Philox blocks of one row");
    chain_row_sites<L, X0, 0, NX / 4>(st, rc, rn, draws, recs, inc, std::make_integer_sequence<int, NX>{});
}

}  // namespace muca
