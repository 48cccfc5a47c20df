// Device side of the counter-based Gaussian generator (see philox.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Philox4x32 round multipliers and Weyl key increments (SC'11, Sect. 4).
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        const uint64_t p0 = (uint64_t)PHILOX_M0 * c[0];
        const uint64_t p1 = (uint64_t)PHILOX_M1 * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// Four FP64 normals for long indices 4q..4q+3 at short index j.
__device__ __forceinline__ void philox_normal4(uint64_t seed, uint32_t tag, uint32_t batch, uint32_t q, uint32_t j,
                                               double z[4]) {
    uint32_t c[4] = {q, j, batch, tag};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double scale = 2.3283064365386963e-10;  // 2^-32
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double ua = ((double)c[2 * h] + 0.5) * scale;
        const double ub = ((double)c[2 * h + 1] + 0.5) * scale;
        const double radius = sqrt(-2.0 * log(ua));
        z[2 * h] = radius * cospi(2.0 * ub);
        z[2 * h + 1] = radius * sinpi(2.0 * ub);
    }
}

// Raw Philox words (used by tests of the generator).
__device__ __forceinline__ void philox_words(uint32_t ctr[4], uint32_t k0, uint32_t k1) { philox4x32_10(ctr, k0, k1); }
