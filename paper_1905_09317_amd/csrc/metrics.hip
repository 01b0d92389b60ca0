// Scar comparison of Section 4 (comparison methodology): per period t the
// simulated scar Y^t (cells whose arrival minute lies in [0, t P]) against a
// reference 0-1 scar X^t, by mean squared error, the structural similarity
// of Wang et al. (2004) over the whole grid (C1 = (0.01 L)^2, C2 =
// (0.03 L)^2, L = 1, N - 1 normalisation; the second denominator factor is
// sigma_x^2 + sigma_y^2 + C2, the printed formula repeating the means there)
// and the Frobenius norm of the last period's difference.
//
// For 0-1 scars every statistic follows from three counts per period: a =
// sum X, b = sum Y, c = sum X Y.  One launch counts them exactly (one 64-bit
// atomic per count and block into a zeroed buffer), and the block that
// finishes last forms the metrics in FP64 from the counts, with the products
// a b, c N and a (N - a) exact in 64-bit integers (N < 2^31), then returns
// the counts and its ticket to zero for the next launch.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernels.h"

namespace c2f {

constexpr int kMetricBlock = 256;
constexpr int kMetricCellsPerThread = 8;

// Metrics of period t from its counts (out[t] = MSE, out[T + t] = SSIM,
// out[2 T] = Frobenius norm of the last period).
__device__ void period_metrics(int64_t a, int64_t b, int64_t c, int t, int T, int64_t n, double* __restrict__ out) {
    const double N = (double)n, N1 = (double)(n - 1);
    const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
    const double mx = (double)a / N, my = (double)b / N;
    const double vx = (double)(a * (n - a)) / (N * N1);
    const double vy = (double)(b * (n - b)) / (N * N1);
    const double cxy = (double)(c * n - a * b) / (N * N1);
    const int64_t diff = a + b - 2 * c;   // cells where the scars differ
    out[t] = (double)diff / N;
    out[T + t] = ((2.0 * mx * my + C1) * (2.0 * cxy + C2)) / ((mx * mx + my * my + C1) * (vx + vy + C2));
    if (t == T - 1) out[2 * T] = sqrt((double)diff);
}

// Every block ends here with partial counts in LDS: part[k] adds to
// counts[base + k] for k < len.  The first wave adds them to the global
// counts, makes its atomics visible
// to the device (release fence) and takes a ticket; the block with the last
// ticket acquires, reads the finished counts, writes the metrics and clears
// counts and ticket for the next launch.  Only the first wave issues global
// atomics, so one release per block suffices; no block waits for another.
__device__ void finish_block(const uint32_t* part, int base, int len, unsigned long long* __restrict__ counts,
                             uint32_t* __restrict__ ticket, int T, int64_t n, double* __restrict__ out) {
    __shared__ bool s_last;
    __syncthreads();
    if (threadIdx.x < 64) {
        for (int k = (int)threadIdx.x; k < len; k += 64)
            if (part[k]) atomicAdd(&counts[base + k], (unsigned long long)part[k]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0) {
            const uint32_t nblocks = gridDim.x * gridDim.y;
            s_last = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nblocks - 1;
        }
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every block's counts are visible from here
    for (int t = (int)threadIdx.x; t < T; t += (int)blockDim.x) {
        unsigned long long v[3];
        for (int f = 0; f < 3; ++f) {
            v[f] = __hip_atomic_load(&counts[3 * t + f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&counts[3 * t + f], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        period_metrics((int64_t)v[0], (int64_t)v[1], (int64_t)v[2], t, T, n, out);
    }
    if (threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// counts[3 t + {0, 1, 2}] += {a, b, c} of period t = blockIdx.y over the
// block's cells.  reference is [T][n]; arrival [n] (-1 = unburned).
__global__ __launch_bounds__(kMetricBlock) void scar_counts_kernel(const int32_t* __restrict__ arrival,
                                                                   const uint8_t* __restrict__ reference,
                                                                   int64_t n, int T, int period_min,
                                                                   unsigned long long* __restrict__ counts,
                                                                   uint32_t* __restrict__ ticket,
                                                                   double* __restrict__ out) {
    const int t = (int)blockIdx.y;
    const int64_t end = (int64_t)(t + 1) * period_min;
    const uint8_t* __restrict__ X = reference + (size_t)t * (size_t)n;
    const int64_t base = (int64_t)blockIdx.x * (kMetricBlock * kMetricCellsPerThread);
    uint32_t a = 0, b = 0, c = 0;   // this wave's counts (valid in every lane)
#pragma unroll
    for (int k = 0; k < kMetricCellsPerThread; ++k) {
        const int64_t i = base + (int64_t)k * kMetricBlock + threadIdx.x;
        bool x = false, y = false;
        if (i < n) {
            x = X[i] != 0;
            const int32_t m = arrival[i];
            y = m >= 0 && (int64_t)m <= end;
        }
        a += (uint32_t)__popcll(__ballot(x));
        b += (uint32_t)__popcll(__ballot(y));
        c += (uint32_t)__popcll(__ballot(x && y));
    }
    __shared__ uint32_t s_cnt[3];
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    if (__lane_id() == 0) {
        atomicAdd(&s_cnt[0], a);
        atomicAdd(&s_cnt[1], b);
        atomicAdd(&s_cnt[2], c);
    }
    finish_block(s_cnt, 3 * t, 3, counts, ticket, T, n, out);
}

// The same counts with every period streamed by each lane over CPL (4 or
// 16) consecutive cells.  Y^t is monotone in t: cell i is in Y^t from its
// burn period k_i = ceil(m_i / P) - 1 on (0 for m_i = 0, never for
// m_i < 0), so each lane computes k_i once.  Periods go in windows of 127:
// with the bytes of kb = min(max(k_i - t_w, 0), 127) for four cells in one
// word, ((t - t_w) * 0x01010101 | 0x80808080) - kb has bit 7 of byte u set
// exactly when cell u is in Y^t (every byte stays in 1..254, so no borrow
// crosses bytes); bit 7 of a byte of (((w & 0x7F..) + 0x7F..) | w) is set
// exactly when that byte of the reference word w is nonzero.  A lane's
// three counts (0..16 each) go packed in 10-bit fields through a DPP sum
// over each 16-lane row (at most 256 per field) and a read of the four row
// sums; wave sums are collected per period in LDS (12 T bytes) and added
// to the global counts once per block.  Reference loads of kRowsBatch
// periods are issued before any is used.  Needs n % CPL == 0, 16-byte
// aligned arrival and CPL-byte aligned reference, T <= kRowsMaxPeriods.
constexpr int kRowsBlock = 1024;
constexpr int kRowsMaxPeriods = 4096;
constexpr int kRowsBatch = 8;
constexpr int kRowsWindow = 127;

__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t w) {
    return (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;
}

// Every lane of each 16-lane row ends with the row's sum: exchanges with
// lane ^ 1 and lane ^ 2 (quad permutations), then the other quad of the
// half row (half mirror), then the other half (mirror).
__device__ __forceinline__ uint32_t row_sum16(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);    // quad_perm 1,0,3,2
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);    // quad_perm 2,3,0,1
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);   // row_half_mirror
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);   // row_mirror
    return v;
}

template <int CPL>
__global__ __launch_bounds__(kRowsBlock) void scar_counts_rows_kernel(const int32_t* __restrict__ arrival,
                                                                      const uint8_t* __restrict__ reference,
                                                                      int64_t q, int T, int period_min,
                                                                      unsigned long long* __restrict__ counts,
                                                                      uint32_t* __restrict__ ticket,
                                                                      double* __restrict__ out) {
    constexpr int W = CPL / 4;   // reference words per lane and period
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    extern __shared__ uint32_t s_cnt[];   // [3 T]
    for (int k = (int)threadIdx.x; k < 3 * T; k += kRowsBlock) s_cnt[k] = 0;
    __syncthreads();
    for (int64_t jb = (int64_t)blockIdx.x * kRowsBlock; jb < q; jb += (int64_t)gridDim.x * kRowsBlock) {
        const int64_t j = jb + threadIdx.x;
        const bool act = j < q;
        int32_t kc[CPL];   // burn period of each of the lane's cells (0x7FFFFFFF = never)
#pragma unroll
        for (int v = 0; v < W; ++v) {
            const int4 m = act ? ((const int4*)arrival)[j * W + v] : make_int4(-1, -1, -1, -1);
            const int32_t mv[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
                kc[4 * v + u] = mv[u] < 0 ? 0x7FFFFFFF : (mv[u] == 0 ? 0 : (mv[u] - 1) / period_min);
        }
        for (int tw = 0; tw < T; tw += kRowsWindow) {
            uint32_t kb[W];
#pragma unroll
            for (int v = 0; v < W; ++v) {
                uint32_t w = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int32_t r = kc[4 * v + u] - tw;
                    w |= (uint32_t)(r < 0 ? 0 : (r > kRowsWindow ? kRowsWindow : r)) << (8 * u);
                }
                kb[v] = w;
            }
            const int tend = min(T, tw + kRowsWindow);
            for (int t0 = tw; t0 < tend; t0 += kRowsBatch) {
                uint32_t wb[kRowsBatch][W];
#pragma unroll
                for (int k = 0; k < kRowsBatch; ++k) {
                    const bool ld = act && t0 + k < tend;
                    if constexpr (W == 4) {
                        u32x4 x = {0u, 0u, 0u, 0u};
                        if (ld) x = ((const u32x4*)reference)[(int64_t)(t0 + k) * q + j];
                        wb[k][0] = x.x;
                        wb[k][1] = x.y;
                        wb[k][2] = x.z;
                        wb[k][3] = x.w;
                    } else {
                        wb[k][0] = ld ? ((const uint32_t*)reference)[(int64_t)(t0 + k) * q + j] : 0u;
                    }
                }
#pragma unroll
                for (int k = 0; k < kRowsBatch; ++k) {
                    const int t = t0 + k;
                    if (t >= tend) break;
                    const uint32_t tb = ((uint32_t)(t - tw) * 0x01010101u) | 0x80808080u;
                    uint32_t ca = 0, cb = 0, cc = 0;
#pragma unroll
                    for (int v = 0; v < W; ++v) {
                        const uint32_t xs = nonzero_bytes(wb[k][v]);
                        const uint32_t ys = (tb - kb[v]) & 0x80808080u;
                        ca += (uint32_t)__popc(xs);
                        cb += (uint32_t)__popc(ys);
                        cc += (uint32_t)__popc(xs & ys);
                    }
                    const uint32_t r = row_sum16(ca | cb << 10 | cc << 20);
                    uint32_t sa = 0, sb = 0, sc = 0;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)r, 16 * g);
                        sa += x & 1023u;
                        sb += (x >> 10) & 1023u;
                        sc += x >> 20;
                    }
                    if (__lane_id() == 0) {
                        if (sa) atomicAdd(&s_cnt[3 * t], sa);
                        if (sb) atomicAdd(&s_cnt[3 * t + 1], sb);
                        if (sc) atomicAdd(&s_cnt[3 * t + 2], sc);
                    }
                }
            }
        }
    }
    finish_block(s_cnt, 0, 3 * T, counts, ticket, T, q * CPL, out);
}

hipError_t launch_scar_metrics(const int32_t* arrival, const uint8_t* reference, int64_t n, int T, int period_min,
                               unsigned long long* counts, uint32_t* ticket, double* out, hipStream_t s) {
    if (n < 2 || T < 1 || T > 65535) return hipErrorInvalidValue;
    const int cpl = (n % 16 == 0 && (uintptr_t)reference % 16 == 0) ? 16
                    : (n % 4 == 0 && (uintptr_t)reference % 4 == 0) ? 4 : 0;
    if (cpl && T <= kRowsMaxPeriods && (uintptr_t)arrival % 16 == 0) {
        const int64_t q = n / cpl;
        const int64_t blocks = std::min<int64_t>((q + kRowsBlock - 1) / kRowsBlock, 2048);
        if (cpl == 16)
            scar_counts_rows_kernel<16><<<(unsigned)blocks, kRowsBlock, (size_t)12 * T, s>>>(
                arrival, reference, q, T, period_min, counts, ticket, out);
        else
            scar_counts_rows_kernel<4><<<(unsigned)blocks, kRowsBlock, (size_t)12 * T, s>>>(
                arrival, reference, q, T, period_min, counts, ticket, out);
    } else {
        const int64_t per_block = (int64_t)kMetricBlock * kMetricCellsPerThread;
        const int64_t gx = (n + per_block - 1) / per_block;
        if (gx * T > 0xFFFFFFFFll) return hipErrorInvalidValue;   // the ticket counts blocks in 32 bits
        const dim3 grid((unsigned)gx, (unsigned)T);
        scar_counts_kernel<<<grid, kMetricBlock, 0, s>>>(arrival, reference, n, T, period_min, counts, ticket, out);
    }
    return hipGetLastError();
}

}  // namespace c2f
