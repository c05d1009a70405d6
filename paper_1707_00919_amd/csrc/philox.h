// philox.h -- Philox4x32-10 for the gfx950 kernels of libmuca.
//
// The counter-based generator the paper picks in Sec. 2.3 (Salmon, Moraes,
// Dror, Shaw, SC'11): ten rounds of two 32x32->64 bit products, the key
// advancing by the two Weyl constants between rounds.  Every walker w uses
// key (seed, w); the counter names the site block and the sweep, so no
// generator state is stored anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muca {

constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeylA = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeylB = 0xBB67AE85u;

struct Words4 {
    uint32_t w[4];
};

// In the sweep the counter words are the same for every lane of a wave and
// only the second key word (the walker) differs, so the first round and half
// of the second are scalar work.  From the third round on every word differs
// per lane; there the two three-input XORs of a round are single gfx950
// v_bitop3_b32 instructions (truth table 0x96 = a ^ b ^ c).
struct PhiloxState {
    uint32_t c0, c1, c2, c3;  // counter, becoming the output
    uint32_t k0, k1;          // key of the next round
};

// Rounds R0 .. R1-1 of a block started with key (k0, k1) at round 0.
template <int R0, int R1>
__device__ __forceinline__ void philox_rounds(PhiloxState& s)
{
#pragma unroll
    for (int round = R0; round < R1; ++round) {
        const uint64_t pa = (uint64_t)kPhiloxMulA * s.c0;
        const uint64_t pb = (uint64_t)kPhiloxMulB * s.c2;
        uint32_t n0, n2;
        if (round < 2) {
            n0 = (uint32_t)(pb >> 32) ^ s.c1 ^ s.k0;
            n2 = (uint32_t)(pa >> 32) ^ s.c3 ^ s.k1;
        } else {
            n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), s.c1, s.k0, 0x96);
            n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), s.c3, s.k1, 0x96);
        }
        s.c1 = (uint32_t)pb;
        s.c3 = (uint32_t)pa;
        s.c0 = n0;
        s.c2 = n2;
        s.k0 += kPhiloxWeylA;
        s.k1 += kPhiloxWeylB;
    }
}

__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1)
{
    PhiloxState s{c0, c1, c2, c3, k0, k1};
    philox_rounds<0, 10>(s);
    return Words4{{s.c0, s.c1, s.c2, s.c3}};
}

}  // namespace muca
