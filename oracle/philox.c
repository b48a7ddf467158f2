/*
 * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
 * published definition: ten rounds of two 32x32->64 multiplies whose high and
 * low halves are mixed with the other counter words and the round key, the key
 * being bumped by the Weyl constants between rounds.
 *
 * The paper relies on fixed randomness for reproducibility (Methodology,
 * reproducibility paragraph); a counter-based stream makes every Monte Carlo
 * draw a pure function of (seed, particle id, step, tag), so the oracle and
 * the GPU can be compared event by event.
 *
 * Counter layout: (id low word, id high word, step, tag << 8 | draw);
 * key: (seed low word, seed high word).
 */
#include "or_internal.h"

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1): the top 23 bits plus one half, times 2^-23.  The result
 * has at most 24 significant bits, so it is exact in single precision too. */
double or_uniform(uint32_t x) {
    return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

void or_draw4(const or_sim *s, uint64_t id, uint32_t step, uint32_t tag, uint32_t draw,
              uint32_t out[4]) {
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, (tag << 8) | draw};
    uint32_t key[2] = {(uint32_t)s->run.seed, (uint32_t)(s->run.seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}
