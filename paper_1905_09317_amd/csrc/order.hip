// Order in which the persistent work groups take the replications of a
// launch that has more replications than resident groups.
//
// A replication's run time is set mostly by the length of its chain of
// dependent propagation passes, which grows with the distance its head fire
// travels (Section 3.4: the head rate of eq. (1) is the fastest axis).  When
// groups take replications in index order, a long replication taken late
// keeps its group busy after every other group has finished.  Taking the
// longest predicted replications first shortens that tail.  The predictor is
// the distance the head fire would cover over the run at the ignition cell's
// own rates: sum over periods of the head rate (with the replication's noise
// draw) times the period length.  The order changes which group runs a
// replication and when, never its result: every replication keeps its index,
// its random streams and its output row, and burn counts are sums.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"
#include "kernels.h"
#include "types.h"

namespace c2f {

// keys[item] += metres the head fire covers in period blockIdx.y at the
// ignition cell's rate; keys start at zero.
template <typename R>
__global__ __launch_bounds__(256) void order_keys_kernel(const Job* __restrict__ jobs, int n_jobs, int total_items,
                                                         unsigned long long* __restrict__ keys) {
    const int item = (int)(blockIdx.x * 256u + threadIdx.x);
    const int p = (int)blockIdx.y;
    if (item >= total_items) return;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].item_base <= item) lo = mid;
        else hi = mid - 1;
    }
    const Job& job = jobs[lo];
    if (p >= job.n_periods || p < job.ign_period || !burning_period(job, p)) return;
    const uint32_t rep = (uint32_t)(job.rep_offset + (item - job.item_base));
    int scen, ign;
    rep_draws(job, rep, scen, ign);
    if (ign < 0 || (int64_t)ign >= (int64_t)job.rows * job.cols) return;
    const CellRec rec = job.cells[ign];
    if (rec_fuel(rec.info) == 0) return;
    RateCtx<R> X;
    X.coef = coef_table<R>();
    X.coef64 = coef_table<double>();
    X.L = land_consts<R>(job.land);
    X.L64 = land_consts<double>(job.land);
    X.rows = (const R*)job.table + (size_t)scen * job.n_wp * kRowLen;
    X.rows64 = job.table64 + (size_t)scen * job.n_wp * kRowLen;
    X.row_stride = kRowLen;
    X.coef32 = coef_table<float>();
    X.L32 = land_consts<float>(job.land);
    X.rows32 = job.table32 ? job.table32 + (size_t)scen * job.n_wp * kRowLen : nullptr;
    X.seed = job.seed;
    X.sigma = (R)job.sigma;
    X.rounding = job.rounding;
    X.rep = rep;
    X.burnout = 0.f;
    X.hfi_min = 0.f;
    const R h = head_rate<R>(X, rec, (uint32_t)ign, (uint32_t)p) * (R)job.period_min;
    // at most 2^20 m per period keeps the sum of up to 2^31 periods in 64 bits
    const unsigned long long v = (h > (R)0) ? (h < (R)1048576 ? (unsigned long long)h : 1048576ull) : 0ull;
    if (v) atomicAdd(&keys[item], v);
}

// Bucket of a key: 32 buckets per octave, larger keys in higher buckets.
constexpr int kOrderBuckets = 64 * 32;

__device__ __forceinline__ int order_bucket(unsigned long long k) {
    if (k == 0) return 0;
    const int msb = 63 - __clzll((long long)k);
    const int frac = msb >= 5 ? (int)((k >> (msb - 5)) & 31ull) : (int)((k << (5 - msb)) & 31ull);
    return msb * 32 + frac;
}

// order[0..total) = the items by decreasing bucket (a counting sort in one
// work group; items of one bucket in no particular order).
__global__ __launch_bounds__(1024) void order_sort_kernel(const unsigned long long* __restrict__ keys,
                                                          int total_items, int32_t* __restrict__ order) {
    __shared__ int s_off[kOrderBuckets];
    for (int b = (int)threadIdx.x; b < kOrderBuckets; b += 1024) s_off[b] = 0;
    __syncthreads();
    for (int i = (int)threadIdx.x; i < total_items; i += 1024) atomicAdd(&s_off[order_bucket(keys[i])], 1);
    __syncthreads();
    // start of each bucket, highest bucket first: a scan over 1024 pairs
    __shared__ int s_part[1024];
    const int b0 = kOrderBuckets - 2 * (int)threadIdx.x - 1;   // this thread's two buckets, descending
    const int c0 = s_off[b0], c1 = s_off[b0 - 1];
    s_part[threadIdx.x] = c0 + c1;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int v = threadIdx.x >= (unsigned)d ? s_part[threadIdx.x - d] : 0;
        __syncthreads();
        s_part[threadIdx.x] += v;
        __syncthreads();
    }
    const int start = s_part[threadIdx.x] - (c0 + c1);   // exclusive
    s_off[b0] = start;
    s_off[b0 - 1] = start + c0;
    __syncthreads();
    for (int i = (int)threadIdx.x; i < total_items; i += 1024) {
        const int pos = atomicAdd(&s_off[order_bucket(keys[i])], 1);
        order[pos] = i;
    }
}

hipError_t launch_order(int precision, const Job* jobs, int n_jobs, int total_items, int max_periods,
                        unsigned long long* keys, int32_t* order, hipStream_t s) {
    if (total_items <= 0) return hipSuccess;
    if (max_periods < 1 || max_periods > 65535) return hipErrorInvalidValue;
    hipError_t e = launch_fill_u32((uint32_t*)keys, (size_t)total_items * 2, 0u, s);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((total_items + 255) / 256), (unsigned)max_periods);
    if (precision == 1)
        order_keys_kernel<float><<<grid, 256, 0, s>>>(jobs, n_jobs, total_items, keys);
    else
        order_keys_kernel<double><<<grid, 256, 0, s>>>(jobs, n_jobs, total_items, keys);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    order_sort_kernel<<<1, 1024, 0, s>>>(keys, total_items, order);
    return hipGetLastError();
}

}  // namespace c2f
