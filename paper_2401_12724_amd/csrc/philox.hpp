// philox.hpp -- the counter-based generator Philox4x32-10 (Salmon, Moraes,
// Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
// Ten rounds; each multiplies counter words 0 and 2 by the round
// multipliers, mixes the high halves with words 1 and 3 and the key, and
// the 2 x 32-bit key advances by the Weyl increments between rounds.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace rng {

__host__ __device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
    const uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
    const uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kWeyl0;
            k1 += kWeyl1;
        }
        uint64_t p0 = (uint64_t)kMul0 * c0;
        uint64_t p1 = (uint64_t)kMul1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// uniform in [0, 1) from the top 24 bits (exact in single precision)
__host__ __device__ inline float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

}  // namespace rng
