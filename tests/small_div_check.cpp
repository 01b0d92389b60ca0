// Host build of ceil_div_small (csrc/small_div.h), checked against integer
// division for every r in [1, 28285] (the longest axis: a diagonal of the
// widest allowed cell) and every q in [1, r + 2], with reciprocals up to two
// ulp off on either side of the correctly rounded 1/q.  Prints the number
// of mismatches and of cases checked.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <initializer_list>

#include "small_div.h"

int main() {
    long bad = 0, n = 0;
    for (int32_t r = 1; r <= 28285; ++r) {
        for (int32_t q = 1; q <= r + 2; ++q) {
            const int32_t want = (r + q - 1) / q;
            float inv = 1.0f / (float)q;
            float lo = std::nextafter(std::nextafter(inv, 0.0f), 0.0f);
            float hi = std::nextafter(std::nextafter(inv, 1.0f), 1.0f);
            for (float v : {lo, inv, hi}) {
                ++n;
                if (c2f::ceil_div_small(r, q, v) != want) {
                    if (bad < 5) std::printf("r=%d q=%d inv=%.9g got %d want %d\n", r, q, v,
                                             c2f::ceil_div_small(r, q, v), want);
                    ++bad;
                }
            }
        }
    }
    std::printf("%ld %ld\n", bad, n);
    return 0;
}
