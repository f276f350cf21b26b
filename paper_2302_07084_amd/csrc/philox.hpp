// Philox4x32-10 counter-based generator for device code (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
// Each round multiplies words 0 and 2 of the counter by the two Philox
// multipliers, exchanges halves and mixes in the key; the key advances by the
// two Weyl increments between rounds.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lne {

// Counter tags (high byte of counter word 3) separating the streams.
constexpr uint32_t kTagEdgeCount = 1u << 24;  // n_e of an edge
constexpr uint32_t kTagWalk = 2u << 24;       // words of one sample slot
constexpr uint32_t kTagOmega = 3u << 24;      // Gaussian test matrix
constexpr uint32_t kTagSparseOmega = 5u << 24; // sparse-sign test matrix

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

}  // namespace lne
