// Host build of the library's FP64 logarithm (csrc/ln64.h) compared with
// the C library's log: prints the largest difference in ulps and the number
// of special-value mismatches.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "ln64.h"

static int64_t ordered(double x) {
    int64_t i;
    std::memcpy(&i, &x, 8);
    return i < 0 ? INT64_MIN - i : i;
}

int main() {
    std::mt19937_64 g(1);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    double worst = 0.0, worst_x = 0.0;
    long n = 0, bad_special = 0;
    auto check = [&](double x) {
        const double a = c2f::ln_f64(x), b = std::log(x);
        if (std::isnan(b) || std::isinf(b)) {
            if (!(std::isnan(a) && std::isnan(b)) && a != b) ++bad_special;
            return;
        }
        const double u = std::fabs((double)(ordered(a) - ordered(b)));
        if (u > worst) {
            worst = u;
            worst_x = x;
        }
        ++n;
    };
    for (int i = 0; i < 500000; ++i) {
        check(std::exp(U(g) * 1380.0 - 690.0));   // the whole normal range
        check(0.5 + 1.5 * U(g));                   // around the range split
        check(0.99 + 0.02 * U(g));                 // near 1
        check(U(g));                               // the rate path's (0, 1)
    }
    const double special[] = {0.0, -0.0, 1.0, 2.0, 0.5, 4.9e-324, 2.2250738585072014e-308,
                              1.7976931348623157e308, -1.0, INFINITY, NAN, 0.7071067811865476,
                              0.7071067811865475, 1.4142135623730951};
    for (double x : special) check(x);
    std::printf("%ld %.17g %.17g %ld\n", n, worst, worst_x, bad_special);
    return 0;
}
