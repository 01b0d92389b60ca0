/* The propagation kernel's ceiling division for the minute an axis reaches
 * its neighbour: t = trunc(r * rcp(q)), then t += (t q < r), for
 * 0 < q < r.  The hardware reciprocal is within one ulp of 1/q, so every
 * r, q pair is checked with the correctly rounded reciprocal and with its
 * neighbours one ulp above and below.  Prints the pairs checked, the
 * failures, and how often the correction was needed. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

static long corrected = 0;

static uint32_t ceil_div(uint32_t r, uint32_t q, float rq) {
    uint32_t t = (uint32_t)((float)r * rq);
    const uint32_t c = (uint32_t)(t * q < r);
    corrected += c;
    return t + c;
}

static long check(uint32_t r, uint32_t q) {
    const float rn = 1.0f / (float)q;
    const float rq[3] = {rn, nextafterf(rn, 0.0f), nextafterf(rn, 2.0f)};
    const uint32_t want = (r + q - 1) / q;
    long bad = 0;
    for (int k = 0; k < 3; ++k) bad += ceil_div(r, q, rq[k]) != want;
    return bad;
}

int main(int argc, char** argv) {
    const uint32_t rmax = argc > 1 ? (uint32_t)atoi(argv[1]) : 28285u;
    long n = 0, bad = 0;
    /* every pair up to rmax (the diagonal of a 20 km cell, in metres) */
    for (uint32_t q = 1; q < rmax; ++q)
        for (uint32_t r = q + 1; r <= rmax; ++r, ++n) bad += check(r, q);
    /* and a sample of pairs up to 2^16 - 1 */
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (int i = 0; i < 20000000; ++i, ++n) {
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        uint32_t a = 1u + (uint32_t)(s % 65535u), b = 1u + (uint32_t)((s >> 32) % 65535u);
        if (a == b) continue;
        bad += check(a > b ? a : b, a > b ? b : a);
    }
    printf("%ld %ld %ld\n", n, bad, corrected);
    return 0;
}
