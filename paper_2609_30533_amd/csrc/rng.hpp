// rng.hpp -- Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and
// Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), device side.
// Ten rounds; each multiplies words 0 and 2 by the Philox constants, swaps the
// halves, xors in the key; the key advances by the Weyl increments between rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace st {

struct U4 {
    uint32_t x[4];
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    U4 r;
    r.x[0] = c0;
    r.x[1] = c1;
    r.x[2] = c2;
    r.x[3] = c3;
    return r;
}

// Top 24 bits scaled to [0, 1): exact in single precision.
__device__ __forceinline__ float unit24f(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }
__device__ __forceinline__ double unit24d(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }
// Uniform integer in [0, n) from the same 24 bits.
__device__ __forceinline__ int32_t index24(uint32_t x, int32_t n) {
    return (int32_t)(((uint64_t)(x >> 8) * (uint64_t)n) >> 24);
}

}  // namespace st
