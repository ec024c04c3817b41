// sk_philox.h -- the counter-based generator of the sketches' random test
// matrices: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11) and Box-Muller normals from its words.
// One definition for every kernel that draws (the projection's Omega, the
// window's power-iteration start vectors and simultaneous-iteration blocks).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

// Ten rounds of Philox4x64 on counter c with key (k0, k1), in place.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t y0 = hi1 ^ c[1] ^ k0;
        const uint64_t y2 = hi0 ^ c[3] ^ k1;
        c[0] = y0;
        c[1] = lo1;
        c[2] = y2;
        c[3] = lo0;
    }
}

// Box-Muller on the word pair (a, b): u1 = ((a >> 11) + 1) 2^-53 in (0, 1],
// u2 = (b >> 11) 2^-53 in [0, 1); cos goes to *n0, sin to *n1.
__device__ __forceinline__ void box_muller(uint64_t a, uint64_t b, double* n0, double* n1) {
    const double u1 = (double)((a >> 11) + 1) * 0x1p-53;
    const double u2 = (double)(b >> 11) * 0x1p-53;
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(6.283185307179586476925286766559 * u2, &sn, &cs);
    *n0 = rad * cs;
    *n1 = rad * sn;
}

// The four N(0,1) draws of counter (c0, c1, c2, c3) under key (seed, stream):
// Box-Muller on words (0, 1) and (2, 3).
__device__ __forceinline__ void gauss4(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1, uint64_t c2,
                                       uint64_t c3, double out[4]) {
    uint64_t c[4] = {c0, c1, c2, c3};
    philox4x64_10(c, seed, stream);
    box_muller(c[0], c[1], &out[0], &out[1]);
    box_muller(c[2], c[3], &out[2], &out[3]);
}

// Draw `which` (0..3) of the same block, computing only its word pair.
__device__ __forceinline__ double gauss_pick(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1, uint64_t c2,
                                             uint64_t c3, int which) {
    uint64_t c[4] = {c0, c1, c2, c3};
    philox4x64_10(c, seed, stream);
    const int h = which >> 1;
    double n0, n1;
    box_muller(c[2 * h], c[2 * h + 1], &n0, &n1);
    return (which & 1) ? n1 : n0;
}

}  // namespace sk
