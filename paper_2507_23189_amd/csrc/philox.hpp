// Philox4x32-10 counter-based generator for the device (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
//
// A round multiplies counter words 0 and 2 by two odd 32-bit constants,
// keeps both halves of each 64-bit product, and permutes them with the
// remaining words and the round key; the key advances by two Weyl constants
// between rounds.  The key here is the run seed (wave-uniform), so the key
// schedule lives in scalar registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcmie {

struct Block4 {
    uint32_t r0, r1, r2, r3;
};

__device__ __forceinline__ Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        // Three-input XOR in one gfx950 instruction (truth table 0x96).
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, k1, 0x96);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return Block4{c0, c1, c2, c3};
}

// Uniform in (0, 1) from one 32-bit word: (2 floor(r / 2^9) + 1) / 2^24,
// exact in FP32 (23 random bits at the centre of their cell).
// Built without a conversion: the 23 bits under the exponent field of 1.0
// give 1 + k 2^-23, and subtracting 1 - 2^-24 is exact (both lie in [1/2, 2]).
__device__ __forceinline__ float uniform01(uint32_t r)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, r, 9u)) - 0x1.fffffep-1f;
}

}  // namespace mcmie
