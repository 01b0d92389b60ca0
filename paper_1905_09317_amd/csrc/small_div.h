// Integer ceiling division on the small operands of the axis stepping.
// Included after <hip/hip_runtime.h>; also compiled for the host by its
// exhaustive test.
#pragma once

#include <stdint.h>

namespace c2f {

// ceil(r / q) for 1 <= r < 2^16 and q >= 1, given inv_q, an approximation
// of 1/q within a few ulp (the hardware reciprocal on the device).  For
// q < r both are below 2^16, so the float quotient r * inv_q is within 0.01
// of r / q and its truncation t is floor(r / q) or one less: the ceiling is
// t, t + 1 or t + 2.  Each test t q < r, exact in float because every
// product here is an integer below 2^18, moves t up by one without passing
// the ceiling.  The general 32-bit division would take a quarter-rate
// multiply sequence per axis.
__host__ __device__ inline int32_t ceil_div_small(int32_t r, int32_t q, float inv_q) {
    if (q >= r) return 1;
    const float fr = (float)r, fq = (float)q;
    float t = (float)(int32_t)(fr * inv_q);
    t += (t * fq < fr) ? 1.0f : 0.0f;
    t += (t * fq < fr) ? 1.0f : 0.0f;
    t += (t * fq < fr) ? 1.0f : 0.0f;
    return (int32_t)t;
}

}  // namespace c2f
