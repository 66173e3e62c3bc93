// Counter-based random numbers on the device: Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011).  A
// 128-bit counter and a 64-bit key give four 32-bit words; each of the ten
// rounds multiplies two counter words by fixed odd constants (full 64-bit
// products), mixes the high halves with the other two words and the key, and
// the key advances by the Weyl constants between rounds.  Stateless: particle n
// of step s draws from counter (n, s, c), so results do not depend on the
// launch shape or the order of the threads.
#pragma once

#include "mcl_internal.h"

namespace mcl {

struct Words4 {
    uint32_t w[4];
};

__device__ inline Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
    constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kW0;
            k1 += kW1;
        }
        const uint32_t hi0 = __umulhi(kM0, c0), lo0 = kM0 * c0;
        const uint32_t hi1 = __umulhi(kM1, c2), lo1 = kM1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return Words4{{c0, c1, c2, c3}};
}

// The 8 words of particle n: counters (n, lo(step), hi(step), c0) and (..., c0 + 1).
__device__ inline void particle_words(uint64_t seed, uint64_t step, uint32_t n, uint32_t c0, uint32_t (&w)[8]) {
    const Words4 a = philox4x32_10(n, (uint32_t)step, (uint32_t)(step >> 32), c0, (uint32_t)seed, (uint32_t)(seed >> 32));
    const Words4 b =
        philox4x32_10(n, (uint32_t)step, (uint32_t)(step >> 32), c0 + 1u, (uint32_t)seed, (uint32_t)(seed >> 32));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        w[i] = a.w[i];
        w[4 + i] = b.w[i];
    }
}

// Uniforms with 24 random bits: (0, 1] and [0, 1).
__device__ inline float unit_open(uint32_t x) { return (float)((x >> 8) + 1u) * 0x1p-24f; }
__device__ inline float unit_closed(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

}  // namespace mcl
