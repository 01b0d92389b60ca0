// Work counts of a finished simulation, recovered from its arrival minutes.
//
// The units of the sending stage (Section 3.8, App. A) as the minute-stepping
// loop of Algorithm 1 meets them:
//   burning-cell-periods  (replication, cell, period) whose rates the cell
//                         takes while some axis still leads to a neighbour
//                         that has not ignited;
//   axis reach events     progress along an axis reaching the neighbour's
//                         centre before that neighbour has ignited;
//   ignitions             burned cells.
// Once every arrival minute is known, each burned cell's own walk is fixed:
// in each period it advances every axis whose neighbour is still available
// (arrival at or after the minute) at its integer rates, so one thread per
// (replication, cell) replays it period by period, with the same rate code
// as the propagation kernel.  Used to measure algorithmic bytes; not on the
// simulation path.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

#include "device.h"
#include "kernels.h"
#include "types.h"

namespace c2f {

template <typename R>
__global__ __launch_bounds__(256) void work_counts_kernel(const Job* __restrict__ jobp,
                                                          const int32_t* __restrict__ arrival,
                                                          unsigned long long* __restrict__ out) {
    __shared__ CoefR<R> s_coef[kNumFuels];
    __shared__ CoefR<double> s_coef64[kNumFuels];
    __shared__ CoefR<float> s_coef32[kNumFuels];
    __shared__ unsigned long long s_sum[3];
    const int tid = threadIdx.x;
    if (tid < kNumFuels) {
        s_coef[tid] = coef_table<R>()[tid];
        s_coef64[tid] = coef_table<double>()[tid];
        s_coef32[tid] = coef_table<float>()[tid];
    }
    if (tid < 3) s_sum[tid] = 0ull;
    __syncthreads();
    const Job& job = *jobp;
    const int64_t n = (int64_t)job.rows * job.cols;
    const int64_t total = n * (int64_t)job.reps;
    const int P = job.period_min;
    const int cols = job.cols;
    const int32_t D[8] = {job.d_orth, job.d_diag, job.d_orth, job.d_diag,
                          job.d_orth, job.d_diag, job.d_orth, job.d_diag};
    const int32_t off[8] = {1, 1 - cols, -cols, -cols - 1, -1, cols - 1, cols, cols + 1};
    unsigned long long c_bp = 0, c_ax = 0, c_ig = 0;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + tid; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = arrival[idx];
        if (a < 0) continue;
        ++c_ig;
        const int64_t r = idx / n;
        const int64_t cell = idx - r * n;
        const CellRec rec = job.cells[cell];
        const uint32_t nb = rec_nbmask(rec.info);
        // final arrival of each in-grid burnable neighbour (INT_MAX: never);
        // -1 marks an axis that never leads anywhere
        int32_t an[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            an[k] = -1;
            if ((nb >> k) & 1u) {
                const int32_t v = arrival[idx + off[k]];
                an[k] = v < 0 ? INT_MAX : v;
            }
        }
        const uint32_t rep = (uint32_t)(job.rep_offset + r);
        int scen = 0, ign = 0;
        rep_draws(job, rep, scen, ign);
        RateCtx<R> X;
        X.coef = s_coef;
        X.coef64 = s_coef64;
        X.L = land_consts<R>(job.land);
        X.L64 = land_consts<double>(job.land);
        X.rows = (const R*)job.table + (size_t)scen * job.n_wp * kRowLen;
        X.rows64 = job.table64 + (size_t)scen * job.n_wp * kRowLen;
        X.row_stride = kRowLen;
        X.coef32 = s_coef32;
        X.L32 = land_consts<float>(job.land);
        X.rows32 = job.table32 ? job.table32 + (size_t)scen * job.n_wp * kRowLen : nullptr;
        X.seed = job.seed;
        X.sigma = (R)job.sigma;
        X.rounding = job.rounding;
        X.rep = rep;
        X.burnout = job.burnout;
        X.hfi_min = job.hfi_min;
        int32_t prog[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        // the cell first spreads in minute a + 1, which lies in period a / P
        for (int p = a / P; p < job.n_periods; ++p) {
            if (!burning_period(job, p)) continue;
            const int32_t ms = max(a + 1, p * P + 1), e = (p + 1) * P;
            if (ms > e) continue;
            bool live = false;
#pragma unroll
            for (int k = 0; k < 8; ++k) live |= an[k] >= ms && prog[k] < D[k];
            if (!live) break;   // no axis can ever become live again
            ++c_bp;
            int32_t q[8];
            if (axis_q<R>(X, rec, (uint32_t)cell, (uint32_t)p, q)) break;   // too faint: burned out
            if (job.burnout > 0.f) {
                int32_t qmax = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if ((nb >> k) & 1u) qmax = max(qmax, q[k]);
                if ((double)qmax < (double)job.burnout) break;   // burned out: spreads no further
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (!(an[k] >= ms && prog[k] < D[k]) || q[k] <= 0) continue;
                // the axis advances q per minute from ms through min(e, an[k])
                // (the neighbour still takes messages in its own arrival minute)
                const int32_t t_end = min(e, an[k]);
                const int32_t need = D[k] - prog[k];
                const int64_t reach = (int64_t)ms + (need + q[k] - 1) / q[k] - 1;
                if (reach <= (int64_t)t_end) {
                    ++c_ax;
                    prog[k] = D[k];
                } else {
                    prog[k] += q[k] * (t_end - ms + 1);   // below need, so no overflow
                }
            }
        }
    }
    atomicAdd(&s_sum[0], c_bp);
    atomicAdd(&s_sum[1], c_ax);
    atomicAdd(&s_sum[2], c_ig);
    __syncthreads();
    if (tid < 3) atomicAdd(&out[tid], s_sum[tid]);
}

hipError_t launch_work_counts(int precision, const Job* job, int64_t total_cells, const int32_t* arrival,
                              unsigned long long* out, hipStream_t s) {
    const int64_t want = (total_cells + 255) / 256;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, 256 * 64));
    if (precision == 1)
        hipLaunchKernelGGL(work_counts_kernel<float>, dim3(grid), dim3(256), 0, s, job, arrival, out);
    else
        hipLaunchKernelGGL(work_counts_kernel<double>, dim3(grid), dim3(256), 0, s, job, arrival, out);
    return hipGetLastError();
}

}  // namespace c2f
