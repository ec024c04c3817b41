/*
 * Counter-based generator for the random matrices the method draws
 * (the Gaussian test matrix of simul_iter, Sec. 2.2, and the Gaussian start
 * vector of the power iteration, Sec. 2.2).  TEST INFRASTRUCTURE ONLY.
 *
 * Philox4x64 with 10 rounds as published by Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC'11): two 64x64->128
 * multiplications per round, the key bumped by the Weyl constants between
 * rounds.  Normals come from the Box-Muller transform on 53-bit uniforms.
 */
#include <math.h>
#include <stdint.h>
#include "oracle.h"

static const uint64_t PH_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PH_M1 = 0xCA5A826395121157ULL;
static const uint64_t PH_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PH_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1  */

static void mul128(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void o_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PH_W0;
            k1 += PH_W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul128(PH_M0, x0, &hi0, &lo0);
        mul128(PH_M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* u in (0, 1]: the top 53 bits plus one, scaled. Never zero, so log is finite. */
static double unit_open0(uint64_t w) { return (double)((w >> 11) + 1) * 0x1p-53; }
/* u in [0, 1). */
static double unit_closed0(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }

void o_gauss4(uint64_t seed, uint64_t stream, const uint64_t ctr[4], double out[4]) {
    const uint64_t key[2] = {seed, stream};
    uint64_t w[4];
    o_philox4x64_10(ctr, key, w);
    const double two_pi = 6.283185307179586476925286766559;
    for (int h = 0; h < 2; ++h) {
        double u1 = unit_open0(w[2 * h]);
        double u2 = unit_closed0(w[2 * h + 1]);
        double rad = sqrt(-2.0 * log(u1));
        double ang = two_pi * u2;
        out[2 * h] = rad * cos(ang);
        out[2 * h + 1] = rad * sin(ang);
    }
}

void o_omega(uint64_t seed, uint64_t stream, uint64_t b, uint64_t tag,
             int d, int k, double* omega) {
    for (int i = 0; i < d; ++i) {
        for (int jg = 0; jg < k; jg += 4) {
            uint64_t ctr[4] = {(uint64_t)i, (uint64_t)(jg >> 2), b, tag};
            double g[4];
            o_gauss4(seed, stream, ctr, g);
            for (int t = 0; t < 4 && jg + t < k; ++t) omega[(int64_t)i * k + jg + t] = g[t];
        }
    }
}
