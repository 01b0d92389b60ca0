// Natural logarithm in FP64 for the rate path.  Included after
// <hip/hip_runtime.h>; the function is also compiled for the host by its
// accuracy test.
#pragma once

#include <cmath>

namespace c2f {

// ln 2 split so that e * kLn2Hi is exact for every binary exponent e
// (kLn2Hi carries 21 significant bits) and kLn2Lo = ln 2 - kLn2Hi.
constexpr double kLn2Hi = 0.6931467056274414;
constexpr double kLn2Lo = 4.7493250390316726e-07;

// ln x from x = m 2^e with m in [sqrt(1/2), sqrt(2)).  With f = m - 1 and
// s = f / (2 + f), ln m = 2 atanh(s) = 2 s (1 + T(s^2)), where T(z) = z/3 +
// z^2/5 + z^3/7 + ... is the Taylor series of atanh(s)/s - 1; |s| <= 0.1716
// makes the tenth term smaller than 2^-53 relative.  Since 2 s = f - s f,
// ln m = f - s (f - 2 T): f is exact and the correction is below f/2, so the
// rounding of s enters only through that correction.  ln x = e ln 2 + ln m
// then rounds about once; the error stays near one ulp (checked against
// libm).  Zero gives -inf, +inf gives +inf, negative or NaN input NaN.
__host__ __device__ inline double ln_f64(double x) {
    const bool finite_pos = x > 0.0 && x < INFINITY;   // false for NaN
    int e = 0;
    double m = frexp(finite_pos ? x : 1.0, &e);   // x = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m += m;
        --e;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double t = 1.0 / 21.0;
    t = fma(t, z, 1.0 / 19.0);
    t = fma(t, z, 1.0 / 17.0);
    t = fma(t, z, 1.0 / 15.0);
    t = fma(t, z, 1.0 / 13.0);
    t = fma(t, z, 1.0 / 11.0);
    t = fma(t, z, 1.0 / 9.0);
    t = fma(t, z, 1.0 / 7.0);
    t = fma(t, z, 1.0 / 5.0);
    t = fma(t, z, 1.0 / 3.0);
    t *= z;
    const double de = (double)e;
    const double r = (de * kLn2Hi + f) - (s * (f - 2.0 * t) - de * kLn2Lo);
    if (finite_pos) return r;
    return (x == 0.0) ? -INFINITY : ((x == INFINITY) ? x : NAN);
}

}  // namespace c2f
