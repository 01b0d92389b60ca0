// gfx950 kernels of the Cell2Fire hot path.
//
//  * landscape preparation: Horn slope numerators, burnable-cell list,
//    nearest-centre burnable cell, landscape constants;
//  * weather table: per (scenario, period) FBP terms that do not depend on
//    the cell;
//  * eval_ros: the per-cell FBP field of one (scenario, period, rep);
//  * propagate: the persistent fire-growth kernel.
//
// Fire growth.  A burning cell i sends fire along each of its 8 axes; after
// it ignites at minute a the fire covers q_k(i, p) metres of axis k in each
// later minute of period p, and reaches neighbour j once the distance D_k is
// covered (Section 3.1, Section 3.4 steps i-ii).  j ignites in that minute
// if its own rate passes the threshold, else at the start of the first later
// period that passes.  Because every hop takes at least one minute and rates
// never depend on arrival order, the arrival minutes are the least solution
// of arrival(j) = min_i next_accept_j(reach_ij(arrival(i))), which the kernel
// finds by label correcting inside one weather period at a time:
//   - each replication runs on one work group, owning an arrival plane
//     (atomicMin on 32-bit labels) and two pairs of work lists;
//   - a cell is processed with its current label: it evaluates the FBP rates
//     for the periods its axes need and walks each axis to the minute it
//     reaches the neighbour (a closed form per period), offering that minute
//     to the neighbour with atomicMin;
//   - improvements inside the current period go to the next round's list,
//     later ones to a future list that is split by period as periods advance;
//   - lists are appended with a wave ballot and prefix count (one LDS atomic
//     per wave), and the period loop stops when no work is left.
// Results are independent of processing order (unique least fixed point).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"
#include "kernels.h"
#include "types.h"

namespace c2f {

// ------------------------------------------------------ coefficient table
__constant__ CoefR<double> kCoef64[kNumFuels] = {C2F_FUEL_ROWS};
__constant__ CoefR<float> kCoef32[kNumFuels] = {C2F_FUEL_ROWS};

template <typename R> __device__ __forceinline__ const CoefR<R>* coef_table();
template <> __device__ __forceinline__ const CoefR<double>* coef_table<double>() { return kCoef64; }
template <> __device__ __forceinline__ const CoefR<float>* coef_table<float>() { return kCoef32; }

template <typename R> __device__ __forceinline__ LandR<R> land_consts(const LandDev* L);
template <> __device__ __forceinline__ LandR<double> land_consts<double>(const LandDev* L) {
    return LandR<double>{L->pc_w64, L->cf64, L->cell_m64};
}
template <> __device__ __forceinline__ LandR<float> land_consts<float>(const LandDev* L) {
    return LandR<float>{L->pc_w32, L->cf32, L->cell_m32};
}

__device__ __forceinline__ int grad_x(uint32_t g) { return (int)(int16_t)(g & 0xFFFFu); }
__device__ __forceinline__ int grad_n(uint32_t g) { return (int)(int16_t)(g >> 16); }

// ------------------------------------------------------------ utilities
__global__ void fill_u32_kernel(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int fill_grid(size_t n) {
    size_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__global__ void fill_tail_kernel(uint8_t* __restrict__ q, int k, uint8_t val) {
    if ((int)threadIdx.x < k) q[threadIdx.x] = val;
}

hipError_t launch_fill_bytes(void* p, size_t bytes, uint8_t v, hipStream_t s) {
    // bulk as 32-bit words (p is at least 4-byte aligned), then the < 4 byte tail
    const uint32_t w = 0x01010101u * v;
    const size_t words = bytes / 4;
    if (words) {
        hipError_t e = launch_fill_u32((uint32_t*)p, words, w, s);
        if (e != hipSuccess) return e;
    }
    const size_t tail = bytes - words * 4;
    if (tail) {
        hipLaunchKernelGGL(fill_tail_kernel, dim3(1), dim3(64), 0, s, (uint8_t*)p + words * 4, (int)tail, v);
        return hipGetLastError();
    }
    return hipSuccess;
}

// -------------------------------------------------- landscape preparation

// Horn's 3x3 gradient numerators with replicated edges:
// gx = east column - west column (weights 1,2,1), gn = north row - south row.
__global__ void grad_kernel(const int16_t* __restrict__ elev, int rows, int cols,
                            uint32_t* __restrict__ grad, int32_t* __restrict__ overflow) {
    const size_t n = (size_t)rows * cols;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / cols), c = (int)(i - (size_t)r * cols);
        const int rn = r > 0 ? r - 1 : 0, rs = r < rows - 1 ? r + 1 : rows - 1;
        const int cw = c > 0 ? c - 1 : 0, ce = c < cols - 1 ? c + 1 : cols - 1;
        auto z = [&](int rr, int cc) { return (int)elev[(size_t)rr * cols + cc]; };
        const int gx = (z(rn, ce) + 2 * z(r, ce) + z(rs, ce)) - (z(rn, cw) + 2 * z(r, cw) + z(rs, cw));
        const int gn = (z(rn, cw) + 2 * z(rn, c) + z(rn, ce)) - (z(rs, cw) + 2 * z(rs, c) + z(rs, ce));
        if (gx > 32767 || gx < -32767 || gn > 32767 || gn < -32767) atomicOr(overflow, 1);
        grad[i] = (uint32_t)(uint16_t)(int16_t)gx | ((uint32_t)(uint16_t)(int16_t)gn << 16);
    }
}

// Burnable-cell list in row-major order: per-tile counts, one-block scan,
// ordered scatter.  A tile is kTile consecutive cells handled by one block.
constexpr int kTileThreads = 256;
constexpr int kTile = kTileThreads * 16;

__global__ void burnable_count_kernel(const uint8_t* __restrict__ fuel, int64_t n,
                                      int32_t* __restrict__ tile_counts) {
    __shared__ int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    int local = 0;
    for (int k = threadIdx.x; k < kTile; k += kTileThreads) {
        const int64_t i = t0 + k;
        local += (i < n && fuel[i] != 0);
    }
    atomicAdd(&s_cnt, local);
    __syncthreads();
    if (threadIdx.x == 0) tile_counts[blockIdx.x] = s_cnt;
}

__global__ void burnable_scan_kernel(int32_t* __restrict__ tile_counts, int n_tiles, LandDev* land) {
    // single block of 1024 threads: exclusive scan in place
    __shared__ int s_part[1024];
    const int per = (n_tiles + 1023) / 1024;
    const int b = threadIdx.x * per;
    int sum = 0;
    for (int k = 0; k < per && b + k < n_tiles; ++k) sum += tile_counts[b + k];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = (threadIdx.x >= (unsigned)off) ? s_part[threadIdx.x - off] : 0;
        __syncthreads();
        s_part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = s_part[threadIdx.x] - sum;   // exclusive prefix of this thread's range
    for (int k = 0; k < per && b + k < n_tiles; ++k) {
        const int c = tile_counts[b + k];
        tile_counts[b + k] = run;
        run += c;
    }
    if (threadIdx.x == 1023) land->n_burnable = s_part[1023];
}

__global__ void burnable_scatter_kernel(const uint8_t* __restrict__ fuel, int64_t n,
                                        const int32_t* __restrict__ tile_offsets,
                                        int32_t* __restrict__ list) {
    __shared__ int s_wave[kTileThreads / 64];
    __shared__ int s_base;
    if (threadIdx.x == 0) s_base = tile_offsets[blockIdx.x];
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k0 = 0; k0 < kTile; k0 += kTileThreads) {
        const int64_t i = t0 + k0 + threadIdx.x;
        const bool b = (i < n) && fuel[i] != 0;
        const uint64_t m = __ballot(b);
        if (lane == 0) s_wave[wave] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < kTileThreads / 64; ++w) {
            if (w < wave) before += s_wave[w];
            total += s_wave[w];
        }
        if (b) {
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            list[s_base + before + rank] = (int32_t)i;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_base += total;
        __syncthreads();
    }
}

// Burnable cell nearest to (rows/2, cols/2); ties go to the lower index.
__global__ void centre_kernel(const uint8_t* __restrict__ fuel, int rows, int cols, LandDev* land) {
    const size_t n = (size_t)rows * cols;
    const int cr = rows / 2, cc = cols / 2;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        if (fuel[i] == 0) continue;
        const long long dr = (long long)(i / cols) - cr, dc = (long long)(i % cols) - cc;
        const unsigned long long key = ((unsigned long long)(dr * dr + dc * dc) << 32) | (unsigned long long)i;
        atomicMin(&land->centre_key, key);
    }
}

// Landscape constants: M-1/M-2 conifer fraction and the O-1 curing factor
// (0.005 (exp(0.061 C) - 1) below 58.8 % curing, 0.176 + 0.02 (C - 58.8) above).
__global__ void landconst_kernel(LandDev* land, float pc, float curing, int cell_m) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double c = (double)curing;
    land->pc_w64 = (double)pc / 100.0;
    land->cf64 = (c < 58.8) ? 0.005 * (exp(0.061 * c) - 1.0) : 0.176 + 0.02 * (c - 58.8);
    land->cell_m64 = (double)cell_m;
    const float cf = curing;
    land->pc_w32 = pc / 100.0f;
    land->cf32 = (cf < 58.8f) ? 0.005f * (expf(0.061f * cf) - 1.0f) : 0.176f + 0.02f * (cf - 58.8f);
    land->cell_m32 = (float)cell_m;
    const unsigned long long key = land->centre_key;
    land->centre_cell = (key == ~0ull) ? -1 : (int32_t)(key & 0xFFFFFFFFull);
}

hipError_t launch_prepare_landscape(const uint8_t* fuel, const int16_t* elev, int rows, int cols,
                                    int cell_m, float pc, float curing, uint32_t* grad,
                                    int32_t* burnable, int32_t* tile_scratch, LandDev* land,
                                    hipStream_t s) {
    const int64_t n = (int64_t)rows * cols;
    const int g = fill_grid((size_t)n);
    hipError_t e;
    // LandDev: zero, then centre key = max
    if ((e = launch_fill_u32((uint32_t*)land, sizeof(LandDev) / 4, 0u, s)) != hipSuccess) return e;
    if ((e = launch_fill_u32((uint32_t*)&land->centre_key, 2, 0xFFFFFFFFu, s)) != hipSuccess) return e;
    if (elev) {
        hipLaunchKernelGGL(grad_kernel, dim3(g), dim3(256), 0, s, elev, rows, cols, grad, &land->grad_overflow);
    } else {
        if ((e = launch_fill_u32(grad, (size_t)n, 0u, s)) != hipSuccess) return e;
    }
    const int n_tiles = (int)((n + kTile - 1) / kTile);
    hipLaunchKernelGGL(burnable_count_kernel, dim3(n_tiles), dim3(kTileThreads), 0, s, fuel, n, tile_scratch);
    hipLaunchKernelGGL(burnable_scan_kernel, dim3(1), dim3(1024), 0, s, tile_scratch, n_tiles, land);
    hipLaunchKernelGGL(burnable_scatter_kernel, dim3(n_tiles), dim3(kTileThreads), 0, s, fuel, n, tile_scratch, burnable);
    hipLaunchKernelGGL(centre_kernel, dim3(g), dim3(256), 0, s, fuel, rows, cols, land);
    hipLaunchKernelGGL(landconst_kernel, dim3(1), dim3(64), 0, s, land, pc, curing, cell_m);
    return hipGetLastError();
}

int64_t tile_scratch_entries(int64_t n_cells) { return (n_cells + kTile - 1) / kTile; }

// ------------------------------------------------------- weather table

template <typename R>
__global__ void weather_table_kernel(const float* __restrict__ wx, int n_rows, R* __restrict__ table) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    const float* w = wx + (size_t)i * 4;
    R row[kRowLen];
    weather_row<R>(coef_table<R>(), w[0], w[1], w[2], w[3], row);
    for (int k = 0; k < kRowLen; ++k) table[(size_t)i * kRowLen + k] = row[k];
}

hipError_t launch_weather_table(const float* wx, int n_rows, double* t64, float* t32, hipStream_t s) {
    const int g = (n_rows + 127) / 128;
    hipLaunchKernelGGL(weather_table_kernel<double>, dim3(g), dim3(128), 0, s, wx, n_rows, t64);
    hipLaunchKernelGGL(weather_table_kernel<float>, dim3(g), dim3(128), 0, s, wx, n_rows, t32);
    return hipGetLastError();
}

// ------------------------------------------- integer axis rates of a cell

// Rates of cell `cell` in period `period`: integer metres per minute along
// the 8 axes (noise applied, then floor(x + u)).
template <typename R>
__device__ __forceinline__ void cell_axis_q(const CoefR<R>* coef, const CoefR<double>* coef64, const LandR<R>& L,
                                            const LandR<double>& L64, int f, uint32_t g, const R* row,
                                            const double* row64, uint64_t seed, uint32_t cell, uint32_t period,
                                            uint32_t rep, R sigma, int rounding, int32_t* q) {
    const CellRates<R> cr = cell_rates<R>(coef, coef64, f, grad_x(g), grad_n(g), row, row64, L, L64);
    const R mu = noise_mult<R>(seed, cell, period, rep, sigma);
    R x[8];
    axis_rates<R>(cr, mu, x);
    R u[8];
    if (rounding == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = (R)0.5;
    } else {
        const uint4 a = draw(seed, cell, period, rep, 1u);
        const uint4 b = draw(seed, cell, period, rep, 2u);
        u[0] = unit24<R>(a.x); u[1] = unit24<R>(a.y); u[2] = unit24<R>(a.z); u[3] = unit24<R>(a.w);
        u[4] = unit24<R>(b.x); u[5] = unit24<R>(b.y); u[6] = unit24<R>(b.z); u[7] = unit24<R>(b.w);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const R v = m_floor(x[k] + u[k]);
        q[k] = (v < (R)1073741824) ? (int32_t)v : 1073741824;
    }
}

// Head rate x noise multiplier of a cell (the receiver's ignition test).
template <typename R>
__device__ __forceinline__ R head_rate(const CoefR<R>* coef, const CoefR<double>* coef64, const LandR<R>& L,
                                       const LandR<double>& L64, int f, uint32_t g, const R* row,
                                       const double* row64, uint64_t seed, uint32_t cell, uint32_t period,
                                       uint32_t rep, R sigma) {
    const CellRates<R> cr = cell_rates<R>(coef, coef64, f, grad_x(g), grad_n(g), row, row64, L, L64);
    return cr.h * noise_mult<R>(seed, cell, period, rep, sigma);
}

// ------------------------------------------------------------- eval_ros

template <typename R>
__global__ void eval_ros_kernel(EvalArgs a) {
    const CoefR<R>* coef = coef_table<R>();
    const CoefR<double>* coef64 = coef_table<double>();
    const LandR<R> L = land_consts<R>(a.land);
    const LandR<double> L64 = land_consts<double>(a.land);
    const size_t ro = ((size_t)a.scenario * a.n_wp + a.period) * kRowLen;
    const R* row = (const R*)a.table + ro;
    const double* row64 = a.table64 + ro;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n_cells; i += gridDim.x * blockDim.x) {
        const int f = a.fuel[i];
        if (f == 0) {
            if (a.hros) a.hros[i] = 0;
            if (a.bros) a.bros[i] = 0;
            if (a.fros) a.fros[i] = 0;
            if (a.lb) a.lb[i] = 0;
            if (a.raz) a.raz[i] = 0;
            for (int k = 0; k < 8; ++k) {
                if (a.x8) a.x8[(size_t)i * 8 + k] = 0;
                if (a.q8) a.q8[(size_t)i * 8 + k] = 0;
            }
            continue;
        }
        const uint32_t g = a.grad[i];
        const CellRates<R> cr = cell_rates<R>(coef, coef64, f, grad_x(g), grad_n(g), row, row64, L, L64);
        const R mu = noise_mult<R>(a.seed, (uint32_t)i, (uint32_t)a.period, a.rep, (R)a.sigma);
        R x[8];
        axis_rates<R>(cr, mu, x);
        int32_t q[8];
        cell_axis_q<R>(coef, coef64, L, L64, f, g, row, row64, a.seed, (uint32_t)i, (uint32_t)a.period, a.rep,
                       (R)a.sigma, a.rounding, q);
        if (a.hros) a.hros[i] = (double)(cr.h * mu);
        if (a.bros) a.bros[i] = (double)(cr.b * mu);
        if (a.fros) a.fros[i] = (double)((cr.h + cr.b) / ((R)2 * cr.lb) * mu);
        if (a.lb) a.lb[i] = (double)cr.lb;
        if (a.raz) {
            double az = 0.0;
            if (cr.wsv > (R)0) {
                az = (double)m_atan2(cr.wx, cr.wy) * (180.0 / 3.14159265358979323846);
                if (az < 0.0) az += 360.0;
            }
            a.raz[i] = az;
        }
        for (int k = 0; k < 8; ++k) {
            if (a.x8) a.x8[(size_t)i * 8 + k] = (double)x[k];
            if (a.q8) a.q8[(size_t)i * 8 + k] = q[k];
        }
    }
}

hipError_t launch_eval_ros(int precision, const EvalArgs& a, hipStream_t s) {
    const int g = fill_grid((size_t)a.n_cells);
    if (precision == 1) hipLaunchKernelGGL(eval_ros_kernel<float>, dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(eval_ros_kernel<double>, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------ propagate

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Append `val` to `list` for every lane with `pred`: one LDS atomic per wave,
// slots assigned by the lane's rank among the wave's appending lanes.
__device__ __forceinline__ void wave_append(bool pred, uint2 val, uint2* __restrict__ list, int* counter,
                                            int64_t cap, int* flag) {
    const uint64_t m = __ballot(pred);
    if (m == 0) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (int)__popcll(m));
    base = __shfl(base, leader);
    if (pred) {
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const int64_t idx = (int64_t)base + rank;
        if (idx < cap) list[idx] = val;
        else *flag = 1;
    }
}

__device__ __forceinline__ uint32_t load_label(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int32_t kNever = 0x7FFFFFFF;

template <typename R, int BLOCK>
__global__ __launch_bounds__(BLOCK) void propagate_kernel(const Job* __restrict__ jobs, int n_jobs,
                                                          int total_items, Slots slots,
                                                          RunCounters* __restrict__ rc) {
    __shared__ int s_item;
    __shared__ int s_nW, s_nWn, s_nF, s_nFn;
    __shared__ int s_flag;
    __shared__ uint32_t s_tag;
    __shared__ int s_scen, s_ign;
    __shared__ unsigned long long s_burned;
    __shared__ unsigned long long s_cnt[kNumCounters];
    __shared__ CoefR<R> s_coef[kNumFuels];
    __shared__ CoefR<double> s_coef64[kNumFuels];

    const int tid = threadIdx.x;
    const int slot = blockIdx.x;
    if (tid < kNumFuels) {
        s_coef[tid] = coef_table<R>()[tid];
        s_coef64[tid] = coef_table<double>()[tid];
    }
    uint32_t* __restrict__ plane = slots.planes + (size_t)slot * (size_t)slots.plane_cells;
    const int64_t cap = slots.list_cap;
    uint2* const listbase = slots.lists + (size_t)slot * 4 * (size_t)cap;

    for (;;) {
        if (tid == 0) {
            int it = atomicAdd(&rc->next_item, 1);
            if (__hip_atomic_load(&rc->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) it = total_items;
            s_item = it;
        }
        __syncthreads();
        const int item = s_item;
        if (item >= total_items) break;

        // job lookup (jobs are sorted by item_base)
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].item_base <= item) lo = mid;
            else hi = mid - 1;
        }
        const Job& job = jobs[lo];
        const int lr = item - job.item_base;
        const uint32_t rep = (uint32_t)(job.rep_offset + lr);
        const int cols = job.cols, rows = job.rows;
        const int P = job.period_min, T = job.T;
        const uint8_t* __restrict__ fuel = job.fuel;
        const uint32_t* __restrict__ grad = job.grad;
        const R* __restrict__ table = (const R*)job.table;
        const LandR<R> L = land_consts<R>(job.land);
        const LandR<double> L64 = land_consts<double>(job.land);
        const R sigma = (R)job.sigma;
        const R thr = (R)job.threshold;
        const bool use_thr = job.threshold > 0.0f;
        const uint64_t seed = job.seed;
        const int rounding = job.rounding;
        const int n_wp = job.n_wp;
        const int32_t D[8] = {job.d_orth, job.d_diag, job.d_orth, job.d_diag,
                              job.d_orth, job.d_diag, job.d_orth, job.d_diag};
        const int DRv[8] = {0, -1, -1, -1, 0, 1, 1, 1};
        const int DCv[8] = {1, 1, 0, -1, -1, -1, 0, 1};

        // ------------------------------------------- replication set-up
        if (tid == 0) {
            uint32_t tag = slots.tags[slot];
            s_tag = tag;   // previous tag; refilled below if exhausted
            s_nW = s_nWn = s_nF = s_nFn = 0;
            s_flag = 0;
            s_burned = 0;
            for (int k = 0; k < kNumCounters; ++k) s_cnt[k] = 0;
            int scen = job.scen_fixed;
            if (job.scen_mode == 1) {
                const uint4 x = draw(seed, 0xFFFFFFFFu, 0xFFFFFFFFu, rep, 4u);
                scen = (int)(((uint64_t)x.x * (uint64_t)job.n_scen) >> 32);
            }
            int ign = -1;
            if (job.ign_mode == 0) {
                ign = job.ign_cell;
            } else if (job.ign_mode == 1) {
                const int nb = job.land->n_burnable;
                if (nb > 0) {
                    const uint4 x = draw(seed, 0xFFFFFFFFu, 0xFFFFFFFFu, rep, 3u);
                    ign = job.burnable[((uint64_t)x.x * (uint64_t)nb) >> 32];
                }
            } else {
                ign = job.land->centre_cell;
            }
            s_scen = scen;
            s_ign = ign;
        }
        __syncthreads();
        if (s_tag <= 1u) {   // tags exhausted: refill this slot's plane
            for (size_t i = tid; i < (size_t)slots.plane_cells; i += BLOCK) plane[i] = kPlaneFill;
            __syncthreads();
            if (tid == 0) s_tag = kTagFresh;
            __syncthreads();
        }
        if (tid == 0) {
            const uint32_t tag = s_tag - 1u;
            s_tag = tag;
            slots.tags[slot] = tag;
            const int ign = s_ign;
            if (ign >= 0 && fuel[ign] != 0) {
                const uint32_t v = tag << kMinuteBits;          // minute 0
                plane[ign] = v;
                listbase[0] = make_uint2((uint32_t)ign, v);
                s_nW = 1;
                s_burned = 1;
                if (job.count) atomicAdd(&job.count[ign], 1u);
            }
        }
        __syncthreads();
        const uint32_t tag = s_tag;
        const int scen = s_scen;
        const R* __restrict__ rows_scen = table + (size_t)scen * n_wp * kRowLen;
        const double* __restrict__ rows64_scen = job.table64 + (size_t)scen * n_wp * kRowLen;

        uint2* curW = listbase;
        uint2* nxtW = listbase + cap;
        uint2* curF = listbase + 2 * cap;
        uint2* nxtF = listbase + 3 * cap;
        unsigned long long c_entries = 0, c_evals = 0, c_cand = 0, c_impr = 0, c_ign = 0;
        int max_list = 0;

        for (int p = 0; p < job.n_periods; ++p) {
            const int32_t e_cur = (p + 1) * P;   // last minute of period p
            if (p > 0) {
                // split the future list: labels in period p -> this period's work list
                const int nF = (int)min((int64_t)s_nF, cap);
                for (int base = 0; base < nF; base += BLOCK) {
                    const int i = base + tid;
                    bool act = i < nF;
                    uint2 ent = make_uint2(0u, 0u);
                    if (act) {
                        ent = curF[i];
                        act = (load_label(&plane[ent.x]) == ent.y);
                    }
                    const int32_t t = (int32_t)(ent.y & kMinuteMask);
                    wave_append(act && t <= e_cur, ent, curW, &s_nW, cap, &s_flag);
                    wave_append(act && t > e_cur, ent, nxtF, &s_nFn, cap, &s_flag);
                }
                __syncthreads();
                if (tid == 0) {
                    s_nF = s_nFn;
                    s_nFn = 0;
                }
                uint2* t2 = curF;
                curF = nxtF;
                nxtF = t2;
                __syncthreads();
            }
            // label-correcting rounds inside period p
            for (;;) {
                const int nW = (int)min((int64_t)s_nW, cap);
                if (nW == 0 || s_flag) break;
                if (nW > max_list) max_list = nW;
                for (int base = 0; base < nW; base += BLOCK) {
                    const int i = base + tid;
                    bool act = i < nW;
                    uint2 ent = make_uint2(0u, 0u);
                    if (act) {
                        ent = curW[i];
                        ++c_entries;
                        act = (load_label(&plane[ent.x]) == ent.y);
                    }
                    const uint32_t c = ent.x;
                    const int32_t a = (int32_t)(ent.y & kMinuteMask);
                    int32_t cand[8], rem[8], curv[8];
                    uint32_t jn[8];
                    uint32_t live = 0;
                    int f = 0;
                    uint32_t g = 0;
                    if (act) {
                        f = fuel[c];
                        g = grad[c];
                        const int r = (int)(c / (uint32_t)cols), col = (int)(c - (uint32_t)r * cols);
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            cand[k] = kNever;
                            rem[k] = D[k];
                            jn[k] = 0;
                            curv[k] = kNever;
                            const int rr = r + DRv[k], cc = col + DCv[k];
                            if (rr < 0 || rr >= rows || cc < 0 || cc >= cols) continue;
                            const uint32_t j = (uint32_t)rr * (uint32_t)cols + (uint32_t)cc;
                            if (fuel[j] == 0) continue;
                            const uint32_t v = plane[j];
                            const int32_t cv = ((v >> kMinuteBits) == tag) ? (int32_t)(v & kMinuteMask) : kNever;
                            if (cv <= a + 1) continue;   // no candidate can beat it
                            jn[k] = j;
                            curv[k] = cv;
                            live |= 1u << k;
                        }
                        // walk the live axes period by period
                        int32_t m0 = a + 1;
                        int pp = a / P;
                        while (live != 0u && m0 <= T) {
                            int32_t q[8];
                            cell_axis_q<R>(s_coef, s_coef64, L, L64, f, g, rows_scen + (size_t)pp * kRowLen,
                                           rows64_scen + (size_t)pp * kRowLen, seed, c, (uint32_t)pp, rep,
                                           sigma, rounding, q);
                            ++c_evals;
                            const int32_t e = min((pp + 1) * P, T);
                            const int64_t n = (int64_t)(e - m0 + 1);
#pragma unroll
                            for (int k = 0; k < 8; ++k) {
                                if (!(live & (1u << k))) continue;
                                const int32_t qk = q[k];
                                if (qk > 0 && (int64_t)qk * n >= rem[k]) {
                                    cand[k] = m0 + (rem[k] + qk - 1) / qk - 1;
                                    live &= ~(1u << k);
                                } else {
                                    rem[k] -= (int32_t)((int64_t)qk * n);
                                    if (curv[k] <= e + 1) live &= ~(1u << k);
                                }
                            }
                            m0 = e + 1;
                            ++pp;
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < 8; ++k) { cand[k] = kNever; jn[k] = 0; }
                    }
                    // offer candidates to the neighbours
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        int32_t t = cand[k];
                        bool has = act && t != kNever;
                        if (has && use_thr) {
                            // ignite at the first minute whose period passes the threshold
                            const uint32_t j = jn[k];
                            const int fj = fuel[j];
                            const uint32_t gj = grad[j];
                            while (t <= T) {
                                const int pj = (t - 1) / P;
                                ++c_evals;
                                if (head_rate<R>(s_coef, s_coef64, L, L64, fj, gj, rows_scen + (size_t)pj * kRowLen,
                                                 rows64_scen + (size_t)pj * kRowLen, seed, j, (uint32_t)pj,
                                                 rep, sigma) > thr)
                                    break;
                                t = (pj + 1) * P + 1;
                            }
                            has = t <= T;
                        }
                        bool improved = false, first = false;
                        uint32_t v = 0;
                        if (has) {
                            ++c_cand;
                            v = (tag << kMinuteBits) | (uint32_t)t;
                            const uint32_t old = atomicMin(&plane[jn[k]], v);
                            improved = v < old;
                            first = improved && ((old >> kMinuteBits) != tag);
                            if (first && job.count) atomicAdd(&job.count[jn[k]], 1u);
                        }
                        c_impr += improved;
                        c_ign += first;
                        wave_append(improved && t <= e_cur, make_uint2(jn[k], v), nxtW, &s_nWn, cap, &s_flag);
                        wave_append(improved && t > e_cur, make_uint2(jn[k], v), curF, &s_nF, cap, &s_flag);
                    }
                }
                __syncthreads();
                if (tid == 0) {
                    s_nW = s_nWn;
                    s_nWn = 0;
                }
                uint2* t2 = curW;
                curW = nxtW;
                nxtW = t2;
                __syncthreads();
            }
            if (s_flag) break;
            if (s_nF == 0) break;   // nothing left to burn
            if (s_nF > max_list) max_list = s_nF;
        }
        if (s_flag && tid == 0) atomicOr(&rc->overflow, 1);

        // per-replication outputs
        atomicAdd(&s_burned, c_ign);
        atomicAdd(&s_cnt[kCntEntries], c_entries);
        atomicAdd(&s_cnt[kCntEvals], c_evals);
        atomicAdd(&s_cnt[kCntCandidates], c_cand);
        atomicAdd(&s_cnt[kCntImprovements], c_impr);
        atomicMax(&s_cnt[kCntMaxList], (unsigned long long)max_list);
        if (job.scar || job.arr_minute || job.arr_period) {
            __syncthreads();
            const size_t n = (size_t)rows * cols;
            const size_t o = (size_t)lr * n;
            for (size_t i = tid; i < n; i += BLOCK) {
                const uint32_t v = load_label(&plane[i]);
                const bool on = (v >> kMinuteBits) == tag;
                const int32_t t = on ? (int32_t)(v & kMinuteMask) : -1;
                if (job.scar) job.scar[o + i] = (uint8_t)on;
                if (job.arr_minute) job.arr_minute[o + i] = t;
                if (job.arr_period) job.arr_period[o + i] = !on ? -1 : (t == 0 ? 0 : (t - 1) / P);
            }
        }
        __syncthreads();
        if (tid == 0) {
            if (job.burned) job.burned[lr] = (int64_t)s_burned;
            s_cnt[kCntIgnitions] = s_burned;
            if (job.ign_out) job.ign_out[lr] = s_ign;
            if (job.scen_out) job.scen_out[lr] = s_scen;
            for (int k = 0; k < kCntMaxList; ++k) atomicAdd(&rc->c[k], s_cnt[k]);
            atomicMax(&rc->c[kCntMaxList], s_cnt[kCntMaxList]);
        }
        __syncthreads();
    }
}

template <typename R>
static hipError_t launch_prop_t(int block, int grid, const Job* jobs, int n_jobs, int total, const Slots& sl,
                                RunCounters* rc, hipStream_t s) {
    switch (block) {
        case 64: hipLaunchKernelGGL((propagate_kernel<R, 64>), dim3(grid), dim3(64), 0, s, jobs, n_jobs, total, sl, rc); break;
        case 128: hipLaunchKernelGGL((propagate_kernel<R, 128>), dim3(grid), dim3(128), 0, s, jobs, n_jobs, total, sl, rc); break;
        case 256: hipLaunchKernelGGL((propagate_kernel<R, 256>), dim3(grid), dim3(256), 0, s, jobs, n_jobs, total, sl, rc); break;
        case 512: hipLaunchKernelGGL((propagate_kernel<R, 512>), dim3(grid), dim3(512), 0, s, jobs, n_jobs, total, sl, rc); break;
        case 1024: hipLaunchKernelGGL((propagate_kernel<R, 1024>), dim3(grid), dim3(1024), 0, s, jobs, n_jobs, total, sl, rc); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_propagate(int precision, int block, int grid, const Job* jobs, int n_jobs, int total,
                            const Slots& slots, RunCounters* rc, hipStream_t s) {
    return precision == 1 ? launch_prop_t<float>(block, grid, jobs, n_jobs, total, slots, rc, s)
                          : launch_prop_t<double>(block, grid, jobs, n_jobs, total, slots, rc, s);
}

template <typename R>
static int occ_t(int block) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (block) {
        case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, propagate_kernel<R, 64>, 64, 0); break;
        case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, propagate_kernel<R, 128>, 128, 0); break;
        case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, propagate_kernel<R, 256>, 256, 0); break;
        case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, propagate_kernel<R, 512>, 512, 0); break;
        case 1024: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, propagate_kernel<R, 1024>, 1024, 0); break;
        default: break;
    }
    return (e == hipSuccess) ? nb : 0;
}

int propagate_blocks_per_cu(int precision, int block) {
    return precision == 1 ? occ_t<float>(block) : occ_t<double>(block);
}

}  // namespace c2f
