// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw, SC 2011), the source
// of the synthetic noise of synth.hip and images.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct Philox4 {
    uint32_t v[4];
};

__host__ __device__ inline void mulhilo32(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
    const uint64_t pr = (uint64_t)a * (uint64_t)b;
    hi = (uint32_t)(pr >> 32);
    lo = (uint32_t)pr;
}

// Philox4x32 with 10 rounds: each round multiplies words 0 and 2 by the round
// multipliers, mixes the high halves with words 1, 3 and the key, and the key is
// bumped by the Weyl constants between rounds.
__host__ __device__ inline Philox4 philox4x32_10(Philox4 c, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(M0, c.v[0], hi0, lo0);
        mulhilo32(M1, c.v[2], hi1, lo1);
        Philox4 n;
        n.v[0] = hi1 ^ c.v[1] ^ k0;
        n.v[1] = lo1;
        n.v[2] = hi0 ^ c.v[3] ^ k1;
        n.v[3] = lo0;
        c = n;
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// Standard normal from one Philox block (Box-Muller on its first two words).
__device__ __forceinline__ float philox_normal(const Philox4& r) {
    const float u1 = ((float)r.v[0] + 0.5f) * 2.3283064365386963e-10f;
    const float u2 = ((float)r.v[1] + 0.5f) * 2.3283064365386963e-10f;
    return sqrtf(-2.f * logf(u1)) * cosf(6.283185307179586f * u2);
}
