// Period-split form of the fire-growth kernel.
//
// For a request whose rates do not depend on the replication (no noise,
// rounding to nearest, one scenario, no ignition threshold), the integer
// axis rates of a cell in a period (FBP rates through eq. (1), Section 3.7)
// are the same for every replication.  The launch then runs one weather
// period at a time: a grid-wide kernel computes the rates of every burnable
// cell in a rectangle around the fire with the whole device, and the period
// kernel (one work group per replication, the same label-correcting work
// queue as the persistent kernel) reads them instead of evaluating; cells
// outside the rectangle are evaluated where they are needed.  Between
// periods a replication's state (generation tag, continuation list and
// counters) lives in global memory; its arrival plane and lists stay in its
// slot.  Results are identical to the persistent kernel's: the same integer
// rates enter the same least-fixed-point computation.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device.h"
#include "kernels.h"
#include "types.h"

namespace c2f {
namespace split {

constexpr int32_t kNever = 0x7FFFFFFF;

__device__ __forceinline__ uint32_t load_label(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int wave_rank(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// One LDS atomic per wave reserves slots for the appending lanes.
__device__ __forceinline__ int wave_reserve(bool pred, int* counter, uint64_t& m) {
    m = __ballot(pred);
    if (m == 0) return 0;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (__lane_id() == leader) base = atomicAdd(counter, (int)__popcll(m));
    return __shfl(base, leader) + wave_rank(m);
}

template <typename T>
__device__ __forceinline__ void append_g(bool pred, const T& val, T* glob, int64_t cap, int* counter, int* flag) {
    uint64_t m;
    const int idx = wave_reserve(pred, counter, m);
    if (pred) {
        if ((int64_t)idx < cap) glob[idx] = val;
        else *flag = 1;
    }
}

// Exclusive prefix sum of `v` over the lanes of a wave, and the wave total.
__device__ __forceinline__ int wave_excl_scan(int v, int& total) {
    const int lane = __lane_id();
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    total = __shfl(x, 63);
    return x - v;
}

// Advance cell c through period p from minute m0 to e (as in the persistent
// kernel), taking the integer rates from qc (8 x u16) when have_q and
// evaluating them otherwise.  max_q collects the largest rate of a live axis.
template <typename R>
__device__ __forceinline__ int advance(const RateCtx<R>& X, const CellRec& rec, uint32_t c, int p, int32_t m0,
                                       int32_t e, const uint32_t* nbv, uint32_t tag, int32_t* rem, int32_t* cand,
                                       bool have_q, const uint4& qc, int32_t& max_q) {
    const uint32_t nb = rec_nbmask(rec.info);
    uint32_t live = 0, settled = 0;   // settled: neighbour label <= e + 1
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        cand[k] = kNever;
        if (!((nb >> k) & 1u) || rem[k] <= 0) {
            rem[k] = 0;
            continue;
        }
        const uint32_t v = nbv[k];
        if ((v >> kMinuteBits) == tag) {
            const int32_t t = (int32_t)(v & kMinuteMask);
            if (t == (int32_t)kPendingMinute || t <= m0) {
                rem[k] = 0;
                continue;
            }
            if (t <= e + 1) settled |= 1u << k;
        }
        live |= 1u << k;
    }
    int evals = 0;
    if (live != 0u && m0 <= e) {
        int32_t q[8];
        if (have_q) {
            const uint32_t w[4] = {qc.x, qc.y, qc.z, qc.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                q[2 * h] = (int32_t)(w[h] & 0xFFFFu);
                q[2 * h + 1] = (int32_t)(w[h] >> 16);
            }
        } else {
            axis_q<R>(X, rec, c, (uint32_t)p, q);
            evals = 1;
        }
        const int64_t n = (int64_t)(e - m0 + 1);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (!((live >> k) & 1u)) continue;
            const int32_t qk = q[k];
            max_q = max(max_q, qk);
            if (qk > 0 && (int64_t)qk * n >= rem[k]) {
                cand[k] = m0 + (rem[k] + qk - 1) / qk - 1;
                rem[k] = 0;
            } else {
                rem[k] -= (int32_t)((int64_t)qk * n);
                if ((settled >> k) & 1u) rem[k] = 0;   // nothing after p can beat it
            }
        }
    }
    return evals;
}

template <int BLOCK>
constexpr int lds_queue_len() {
    return 2 * (BLOCK <= 64 ? 512 : (BLOCK <= 128 ? 1024 : (BLOCK <= 256 ? 2048 : 4096)));
}

}  // namespace split

__global__ void split_region_init_kernel(SplitRegion* reg) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        reg->r0 = reg->c0 = 0x7FFFFFFF;
        reg->r1 = reg->c1 = -1;
        reg->max_q[0] = reg->max_q[1] = 0;
        reg->cr0 = reg->cc0 = 0;
        reg->cr1 = reg->cc1 = -1;
    }
}

// Replication set-up: scenario and ignition draws, the slot's next
// generation tag (refilling its plane when they run out), the ignition at
// minute 0 as a continuation of period 0 with every axis at full distance.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void split_setup_kernel(const Job* __restrict__ jobs, int total_items, Slots slots,
                                                            SplitState* __restrict__ st,
                                                            SplitRegion* __restrict__ reg) {
    __shared__ uint32_t s_tag;
    const int tid = threadIdx.x;
    const int item = blockIdx.x;
    if (item >= total_items) return;
    const Job& job = jobs[0];
    const uint32_t rep = (uint32_t)(job.rep_offset + item);
    uint32_t* __restrict__ plane = slots.planes + (size_t)item * (size_t)slots.plane_cells;
    if (tid == 0) s_tag = slots.tags[item];
    __syncthreads();
    if (s_tag <= 1u) {   // tags exhausted: refill this slot's plane
        for (size_t i = tid; i < (size_t)slots.plane_cells; i += BLOCK) plane[i] = kPlaneFill;
        __syncthreads();
        if (tid == 0) s_tag = kTagFresh;
        __syncthreads();
    }
    if (tid != 0) return;
    const uint32_t tag = s_tag - 1u;
    slots.tags[item] = tag;
    int scen = job.scen_fixed;
    if (job.scen_mode == 1) {
        const uint4 x = draw(job.seed, 0xFFFFFFFFu, 0xFFFFFFFFu, rep, 4u);
        scen = (int)(((uint64_t)x.x * (uint64_t)job.n_scen) >> 32);
    }
    int ign = -1;
    if (job.ign_mode == 0) {
        ign = job.ign_cell;
    } else if (job.ign_mode == 1) {
        const int nbn = job.land->n_burnable;
        if (nbn > 0) {
            const uint4 x = draw(job.seed, 0xFFFFFFFFu, 0xFFFFFFFFu, rep, 3u);
            ign = job.burnable[((uint64_t)x.x * (uint64_t)nbn) >> 32];
        }
    } else {
        ign = job.land->centre_cell;
    }
    SplitState s;
    s.tag = tag;
    s.cc = 0;
    s.nC = 0;
    s.flag = 0;
    s.scen = scen;
    s.ign = ign;
    s.max_list = 0;
    for (int k = 0; k < 8; ++k) s.cnt[k] = 0;
    if (ign >= 0 && rec_fuel(job.cells[ign].info) != 0) {
        const uint32_t v = tag << kMinuteBits;   // minute 0
        plane[ign] = v;
        const int64_t stride = slots.list_cap;
        Cont* gC0 = (Cont*)(slots.lists + (size_t)item * (size_t)stride * (size_t)kSlotListBytesPerEntry + 16 * stride);
        Cont ct;
        ct.c = (uint32_t)ign;
        ct.label = v;
        const uint32_t dd = (uint32_t)job.d_orth | ((uint32_t)job.d_diag << 16);
        for (int h = 0; h < 4; ++h) ct.rem[h] = dd;   // E/N/W/S full, NE/NW/SW/SE full
        gC0[0] = ct;
        s.nC = 1;
        s.cnt[kCntIgnitions] = 1;
        if (job.count) atomicAdd(&job.count[ign], 1u);
        const int r = ign / job.cols, c = ign - r * job.cols;
        atomicMin(&reg->r0, r);
        atomicMax(&reg->r1, r);
        atomicMin(&reg->c0, c);
        atomicMax(&reg->c1, c);
    }
    s.done = s.nC == 0;
    st[item] = s;
}

// Integer axis rates of period p for every burnable cell in the rectangle
// around the fire: the bounding box of the cells ignited so far widened by
// the distance the last period's fastest axis covers in 1.5 periods (32
// cells before the first period).
template <typename R>
__global__ __launch_bounds__(256) void rate_region_kernel(const Job* __restrict__ jobs, SplitRegion* __restrict__ reg,
                                                          uint4* __restrict__ cache, int p) {
    __shared__ CoefR<R> s_coef[kNumFuels];
    __shared__ CoefR<double> s_coef64[kNumFuels];
    const int tid = threadIdx.x;
    if (tid < kNumFuels) {
        s_coef[tid] = coef_table<R>()[tid];
        s_coef64[tid] = coef_table<double>()[tid];
    }
    __syncthreads();
    const Job& job = jobs[0];
    const int rows = job.rows, cols = job.cols;
    const int b_r0 = reg->r0, b_r1 = reg->r1, b_c0 = reg->c0, b_c1 = reg->c1;
    if (b_r1 < b_r0) return;   // nothing burns
    const int32_t mq = p > 0 ? reg->max_q[(p - 1) & 1] : 0;
    int margin = 32;
    if (mq > 0) {
        const int64_t m = ((int64_t)mq * job.period_min * 3 / 2 + job.d_orth - 1) / job.d_orth + 2;
        margin = (int)std::min<int64_t>(std::max<int64_t>(m, 8), 512);
    }
    const int r0 = max(0, b_r0 - margin), r1 = min(rows - 1, b_r1 + margin);
    const int c0 = max(0, b_c0 - margin), c1 = min(cols - 1, b_c1 + margin);
    if (blockIdx.x == 0 && tid == 0) {
        reg->cr0 = r0;
        reg->cr1 = r1;
        reg->cc0 = c0;
        reg->cc1 = c1;
        reg->max_q[p & 1] = 0;   // collected by this period's kernel
    }
    RateCtx<R> X;
    X.coef = s_coef;
    X.coef64 = s_coef64;
    X.L = land_consts<R>(job.land);
    X.L64 = land_consts<double>(job.land);
    X.rows = (const R*)job.table + (size_t)job.scen_fixed * job.n_wp * kRowLen;
    X.rows64 = job.table64 + (size_t)job.scen_fixed * job.n_wp * kRowLen;
    X.seed = job.seed;
    X.sigma = (R)0;
    X.rounding = 0;
    X.rep = 0;
    const int w = c1 - c0 + 1;
    const int64_t n = (int64_t)(r1 - r0 + 1) * w;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + tid; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int dr = (int)(i / w);
        const int r = r0 + dr, c = c0 + (int)(i - (int64_t)dr * w);
        const uint32_t cell = (uint32_t)r * (uint32_t)cols + (uint32_t)c;
        const CellRec rec = job.cells[cell];
        if (rec_fuel(rec.info) == 0) continue;
        int32_t q[8];
        axis_q<R>(X, rec, cell, (uint32_t)p, q);
        uint32_t wq[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            // a rate of the longest axis distance or more reaches the
            // neighbour in one minute either way: 16 bits keep every outcome
            const uint32_t a = (uint32_t)min(q[2 * h], 65535), b = (uint32_t)min(q[2 * h + 1], 65535);
            wq[h] = a | (b << 16);
        }
        cache[cell] = make_uint4(wq[0], wq[1], wq[2], wq[3]);
    }
}

// One weather period of every replication of the launch (item i in slot i).
template <typename R, int BLOCK>
__global__ __launch_bounds__(BLOCK, 2) void split_period_kernel(const Job* __restrict__ jobs, int total_items,
                                                             Slots slots, SplitState* __restrict__ st,
                                                             SplitRegion* __restrict__ reg,
                                                             const uint4* __restrict__ cache, int p) {
    using namespace split;
    constexpr int LQ = lds_queue_len<BLOCK>();
    __shared__ uint2 s_Q[LQ];
    __shared__ int s_res, s_commit;   // queue entries reserved, committed (in order)
    // queue entries taken (high 32 bits) and waves holding a chunk (low 32)
    __shared__ unsigned long long s_hb;
    __shared__ int s_nC[2];
    __shared__ int s_flag, s_done;
    __shared__ int s_r0, s_r1, s_c0, s_c1, s_maxq;
    __shared__ unsigned long long s_cnt[kNumCounters];
    __shared__ CoefR<R> s_coef[kNumFuels];
    __shared__ CoefR<double> s_coef64[kNumFuels];

    const int tid = threadIdx.x;
    const int item = blockIdx.x;
    if (item >= total_items) return;
    SplitState* __restrict__ me = &st[item];
    if (tid == 0) s_done = me->done;
    if (tid < kNumFuels) {
        s_coef[tid] = coef_table<R>()[tid];
        s_coef64[tid] = coef_table<double>()[tid];
    }
    __syncthreads();
    if (s_done) return;   // the fire is out (or overflowed) in this replication
    const Job& job = jobs[0];
    const uint32_t rep = (uint32_t)(job.rep_offset + item);
    const int cols = job.cols;
    const int rows = job.rows;
    const int P = job.period_min;
    const CellRec* __restrict__ cells = job.cells;
    const int32_t D[8] = {job.d_orth, job.d_diag, job.d_orth, job.d_diag,
                          job.d_orth, job.d_diag, job.d_orth, job.d_diag};
    const int32_t off[8] = {1, 1 - cols, -cols, -cols - 1, -1, cols - 1, cols, cols + 1};
    uint32_t* __restrict__ plane = slots.planes + (size_t)item * (size_t)slots.plane_cells;
    const int64_t stride = slots.list_cap;
    const int64_t cap = slots.list_limit;
    uint8_t* lb = slots.lists + (size_t)item * (size_t)stride * (size_t)kSlotListBytesPerEntry;
    uint2* const gQ = (uint2*)lb;   // global part of the period queue: 2 x cap entries
    Cont* const gC0 = (Cont*)(lb + 16 * stride);
    const int cc = me->cc;
    Cont* const gCin = gC0 + (size_t)cc * stride;
    Cont* const gCout = gC0 + (size_t)(cc ^ 1) * stride;
    const uint32_t tag = me->tag;
    const int scen = me->scen;
    if (tid == 0) {
        s_res = s_commit = 0;
        s_hb = 0ull;
        s_nC[0] = me->nC;   // continuations in
        s_nC[1] = 0;        // continuations out
        s_flag = 0;
        for (int k = 0; k < kNumCounters; ++k) s_cnt[k] = 0;
        s_r0 = s_c0 = 0x7FFFFFFF;
        s_r1 = s_c1 = -1;
        s_maxq = 0;
    }
    RateCtx<R> X;
    X.coef = s_coef;
    X.coef64 = s_coef64;
    X.L = land_consts<R>(job.land);
    X.L64 = land_consts<double>(job.land);
    X.rows = (const R*)job.table + (size_t)scen * job.n_wp * kRowLen;
    X.rows64 = job.table64 + (size_t)scen * job.n_wp * kRowLen;
    X.seed = job.seed;
    X.sigma = (R)job.sigma;
    X.rounding = job.rounding;
    X.rep = rep;
    X.burnout = 0.f;
    const int rr0 = reg->cr0, rr1 = reg->cr1, rc0 = reg->cc0, rc1 = reg->cc1;   // cached rectangle
    const int32_t s = p * P + 1;     // first minute of period p
    const int32_t e = (p + 1) * P;   // last minute of period p
    const int64_t qcap = (int64_t)LQ + 2 * cap;
    __syncthreads();

    uint32_t c_entries = 0, c_conts = 0, c_evals = 0, c_cand = 0, c_impr = 0, c_ign = 0, c_chunks = 0;
    int32_t max_q = 0;
    int b_r0 = 0x7FFFFFFF, b_r1 = -1, b_c0 = 0x7FFFFFFF, b_c1 = -1;

    // Commit a reserved queue range in reservation order (earlier
    // reservations never wait on later ones); wave-uniform control flow.
    auto q_commit = [&](int wbase, int wtot) __attribute__((always_inline)) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (__lane_id() == 0) {
            while (__hip_atomic_load(&s_commit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != wbase)
                __builtin_amdgcn_s_sleep(1);
            __hip_atomic_store(&s_commit, wbase + wtot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };

    // Advance one entry per lane (a continuation from the start of p, or an
    // improved cell from its minute); improvements go to the queue, axes
    // still travelling at the end of p to the outgoing continuation list.
    auto process = [&](bool act, uint32_t c, uint32_t lab, int32_t* rem, bool conts) __attribute__((always_inline)) {
        int32_t cand[8];
        uint32_t nbv[8];
        CellRec rec;
        rec.info = 0;
        uint4 qc = make_uint4(0u, 0u, 0u, 0u);
        bool have_q = false;
        int r = 0, col = 0;
        if (act) {
            // every load of the entry at once: own label, cell record, cached
            // rates and the labels of the in-grid neighbours
            const uint32_t own = load_label(&plane[c]);
            rec = cells[c];
            r = (int)(c / (uint32_t)cols);
            col = (int)(c - (uint32_t)r * (uint32_t)cols);
            have_q = r >= rr0 && r <= rr1 && col >= rc0 && col <= rc1;
            if (have_q) qc = cache[c];
            uint32_t inb = 0xFFu;
            if (col + 1 >= cols) inb &= ~0x83u;   // E, NE, SE
            if (col == 0) inb &= ~0x38u;          // NW, W, SW
            if (r == 0) inb &= ~0x0Eu;            // NE, N, NW
            if (r + 1 >= rows) inb &= ~0xE0u;     // SW, S, SE
#pragma unroll
            for (int k = 0; k < 8; ++k) nbv[k] = ((inb >> k) & 1u) ? plane[(int64_t)c + off[k]] : kPlaneFill;
            act = own == lab;
        }
        bool keep = false;
        if (act) {
            const int32_t m0 = conts ? s : (int32_t)(lab & kMinuteMask) + 1;
            c_evals += advance<R>(X, rec, c, p, m0, e, nbv, tag, rem, cand, have_q, qc, max_q);
            keep = (rem[0] | rem[1] | rem[2] | rem[3] | rem[4] | rem[5] | rem[6] | rem[7]) != 0;
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                cand[k] = kNever;
                rem[k] = 0;
            }
        }
        // offer the candidates with atomicMin, all issued before any is used
        uint32_t hasm = 0, impr = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) hasm |= (act && cand[k] != kNever) ? (1u << k) : 0u;
        uint32_t old[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            old[k] = 0u;
            if ((hasm >> k) & 1u) old[k] = atomicMin(&plane[(int64_t)c + off[k]], (tag << kMinuteBits) | (uint32_t)cand[k]);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (!((hasm >> k) & 1u)) continue;
            const uint32_t v = (tag << kMinuteBits) | (uint32_t)cand[k];
            if (v < old[k]) {
                impr |= 1u << k;
                if ((old[k] >> kMinuteBits) != tag || (old[k] & kMinuteMask) == kPendingMinute) {
                    ++c_ign;
                    if (job.count) atomicAdd(&job.count[(int64_t)c + off[k]], 1u);
                }
            }
        }
        c_cand += __popc(hasm);
        if (impr != 0u) {
            // rows and columns reached by the improved axes
            b_r0 = min(b_r0, r - ((impr & 0x0Eu) ? 1 : 0));
            b_r1 = max(b_r1, r + ((impr & 0xE0u) ? 1 : 0));
            b_c0 = min(b_c0, col - ((impr & 0x38u) ? 1 : 0));
            b_c1 = max(b_c1, col + ((impr & 0x83u) ? 1 : 0));
        }
        // append this lane's improved neighbours with one wave scan
        const int ni = __popc(impr);
        c_impr += ni;
        int wtot;
        const int pre = wave_excl_scan(ni, wtot);
        if (wtot > 0) {
            int wbase = 0;
            if (__lane_id() == 0) wbase = atomicAdd(&s_res, wtot);
            wbase = __shfl(wbase, 0);
            int idx = wbase + pre;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (!((impr >> k) & 1u)) continue;
                const uint2 val = make_uint2((uint32_t)((int64_t)c + off[k]), (tag << kMinuteBits) | (uint32_t)cand[k]);
                if (idx < LQ) s_Q[idx] = val;
                else if ((int64_t)(idx - LQ) < 2 * cap) gQ[idx - LQ] = val;
                else s_flag = 1;
                ++idx;
            }
            q_commit(wbase, wtot);
        }
        Cont ct;
        ct.c = c;
        ct.label = lab;
#pragma unroll
        for (int h = 0; h < 4; ++h) ct.rem[h] = (uint32_t)rem[2 * h] | ((uint32_t)rem[2 * h + 1] << 16);
        append_g(keep, ct, gCout, cap, &s_nC[1], &s_flag);
    };

    // continuations of p-1, advanced from the start of p
    {
        const int n = (int)min((int64_t)s_nC[0], cap);
        for (int base = 0; base < n; base += BLOCK) {
            const int i = base + tid;
            const bool act = i < n;
            uint32_t c = 0, lab = 0;
            int32_t rem[8];
            if (act) {
                const Cont ct = gCin[i];
                c = ct.c;
                lab = ct.label;
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    rem[2 * h] = (int32_t)(ct.rem[h] & 0xFFFFu);
                    rem[2 * h + 1] = (int32_t)(ct.rem[h] >> 16);
                }
                ++c_conts;
            }
            process(act, c, lab, rem, true);
        }
    }
    __syncthreads();

    // label correcting over the period's queue
    for (;;) {
        int base = 0, cnt = 0;
        bool done = false;
        if (__lane_id() == 0) {
            for (;;) {
                if (__hip_atomic_load(&s_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                    done = true;
                    break;
                }
                const unsigned long long hb = __hip_atomic_load(&s_hb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const int h = (int)(hb >> 32), holders = (int)(uint32_t)hb;
                const int cm = __hip_atomic_load(&s_commit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (h < cm) {
                    const int take = min(64, cm - h);
                    const unsigned long long nhb = ((unsigned long long)(uint32_t)(h + take) << 32) |
                                                   (unsigned long long)(uint32_t)(holders + 1);
                    if (atomicCAS(&s_hb, hb, nhb) == hb) {
                        base = h;
                        cnt = take;
                        break;
                    }
                    continue;
                }
                // finished when no wave holds a chunk (so none can append)
                // and every reserved entry has been taken
                const int rs = __hip_atomic_load(&s_res, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (holders == 0 && h == cm && cm == rs) {
                    done = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        base = __shfl(base, 0);
        cnt = __shfl(cnt, 0);
        done = __shfl((int)done, 0) != 0;
        if (done) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        ++c_chunks;
        const int i = base + __lane_id();
        const bool act = __lane_id() < cnt && (int64_t)i < qcap;
        uint32_t c = 0, lab = 0;
        int32_t rem[8];
        if (act) {
            uint2 ent;
            if (i < LQ) {
                ent = s_Q[i];
            } else {
                const uint64_t v = __hip_atomic_load((const uint64_t*)&gQ[i - LQ], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                ent = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
            }
            c = ent.x;
            lab = ent.y;
#pragma unroll
            for (int k = 0; k < 8; ++k) rem[k] = D[k];
            ++c_entries;
        }
        process(act, c, lab, rem, false);
        if (__lane_id() == 0) atomicAdd(&s_hb, ~0ull);   // one holder fewer
    }

    // period end: fold the tallies and save the replication's state
    atomicAdd(&s_cnt[kCntIgnitions], (unsigned long long)c_ign);
    atomicAdd(&s_cnt[kCntEntries], (unsigned long long)c_entries);
    atomicAdd(&s_cnt[kCntConts], (unsigned long long)c_conts);
    atomicAdd(&s_cnt[kCntEvals], (unsigned long long)c_evals);
    atomicAdd(&s_cnt[kCntCandidates], (unsigned long long)c_cand);
    atomicAdd(&s_cnt[kCntImprovements], (unsigned long long)c_impr);
    if (__lane_id() == 0) atomicAdd(&s_cnt[kCntRounds], (unsigned long long)c_chunks);
    atomicMin(&s_r0, b_r0);
    atomicMax(&s_r1, b_r1);
    atomicMin(&s_c0, b_c0);
    atomicMax(&s_c1, b_c1);
    atomicMax(&s_maxq, max_q);
    __syncthreads();
    if (tid == 0) {
        SplitState sv = *me;
        sv.cc = cc ^ 1;
        sv.nC = s_nC[1];
        sv.flag |= s_flag;
        sv.done = sv.flag || sv.nC == 0 || p + 1 >= job.n_periods;
        const int ml = max(max(s_nC[0], s_nC[1]), s_res);
        sv.max_list = max(sv.max_list, ml);
        for (int k = 0; k < kCntMaxList; ++k) sv.cnt[k] += (uint32_t)s_cnt[k];
        *me = sv;
        if (s_r1 >= s_r0) {
            atomicMin(&reg->r0, s_r0);
            atomicMax(&reg->r1, s_r1);
            atomicMin(&reg->c0, s_c0);
            atomicMax(&reg->c1, s_c1);
        }
        atomicMax(&reg->max_q[p & 1], s_maxq);
    }
}

// Per-replication outputs and counters of a period-split launch.
__global__ void split_finish_kernel(const Job* __restrict__ jobs, int total_items, Slots slots,
                                    const SplitState* __restrict__ st, RunCounters* __restrict__ rc) {
    const int item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= total_items) return;
    const Job& job = jobs[0];
    const SplitState s = st[item];
    if (s.flag) atomicOr(&rc->overflow, 1);
    for (int k = 0; k < kCntMaxList; ++k) atomicAdd(&rc->c[k], (unsigned long long)s.cnt[k]);
    atomicMax(&rc->c[kCntMaxList], (unsigned long long)s.max_list);
    if (job.burned) job.burned[item] = (int64_t)s.cnt[kCntIgnitions];
    if (job.ign_out) job.ign_out[item] = s.ign;
    if (job.scen_out) job.scen_out[item] = s.scen;
    if (slots.item_slot) slots.item_slot[item] = make_int2(item, (int)s.tag);
}

#define C2F_SPLIT_BLOCKS(block, CALL)         \
    switch (block) {                          \
        case 64: CALL(64); break;             \
        case 128: CALL(128); break;           \
        case 256: CALL(256); break;           \
        case 512: CALL(512); break;           \
        case 1024: CALL(1024); break;         \
        default: return hipErrorInvalidValue; \
    }

template <typename R>
static hipError_t launch_split_t(int block, const Job* jobs, int total, int n_periods, int rate_blocks,
                                 const Slots& sl, SplitState* st, SplitRegion* reg, uint4* cache, RunCounters* rc,
                                 hipStream_t s) {
    hipLaunchKernelGGL(split_region_init_kernel, dim3(1), dim3(64), 0, s, reg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define C2F_SETUP(B) hipLaunchKernelGGL((split_setup_kernel<B>), dim3(total), dim3(B), 0, s, jobs, total, sl, st, reg)
    C2F_SPLIT_BLOCKS(block, C2F_SETUP)
#undef C2F_SETUP
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int p = 0; p < n_periods; ++p) {
        hipLaunchKernelGGL((rate_region_kernel<R>), dim3(rate_blocks), dim3(256), 0, s, jobs, reg, cache, p);
        if ((e = hipGetLastError()) != hipSuccess) return e;
#define C2F_PERIOD(B) \
    hipLaunchKernelGGL((split_period_kernel<R, B>), dim3(total), dim3(B), 0, s, jobs, total, sl, st, reg, cache, p)
        C2F_SPLIT_BLOCKS(block, C2F_PERIOD)
#undef C2F_PERIOD
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(split_finish_kernel, dim3((total + 255) / 256), dim3(256), 0, s, jobs, total, sl, st, rc);
    return hipGetLastError();
}

#undef C2F_SPLIT_BLOCKS

hipError_t launch_split(int precision, int block, const Job* jobs, int total, int n_periods, int rate_blocks,
                        const Slots& slots, SplitState* st, SplitRegion* reg, uint4* cache, RunCounters* rc,
                        hipStream_t s) {
    return precision == 1
               ? launch_split_t<float>(block, jobs, total, n_periods, rate_blocks, slots, st, reg, cache, rc, s)
               : launch_split_t<double>(block, jobs, total, n_periods, rate_blocks, slots, st, reg, cache, rc, s);
}

}  // namespace c2f
