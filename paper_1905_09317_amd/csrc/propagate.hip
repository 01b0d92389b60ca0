// The persistent fire-growth kernel.
//
// Model (Sections 3.1 and 3.4, Algorithm 1 Step 2).  Once a cell ignites at
// minute a, its fire advances q_k(p) metres along axis k in each later minute
// of period p (the FBP rates of the cell in that period through eq. (1)),
// and reaches neighbour k once the distance D_k between the two centres is
// covered.  The neighbour ignites in that minute if its own head rate passes
// the threshold, else at the start of the first later period that passes
// (the message persists).  Every hop takes at least one minute and rates do
// not depend on the order of ignitions, so the arrival minutes are the least
// solution of arrival(j) = min_i accept_j(reach_ij(arrival(i))): any
// evaluation order that only commits arrivals of the current period and
// carries per-axis progress across period ends gives exactly the minute-
// stepping result.
//
// Work decomposition.  One work group per replication (persistent groups
// take replications from a counter).  Per weather period p:
//   - cells waiting for a passing rate (pending) are re-tested;
//   - cells whose axes were still travelling at the end of p-1
//     (continuations, with the metres left on each axis) are advanced
//     through p, those listed last (lit latest, at the fire front) first;
//   - label correcting: each cell that received a smaller arrival in p is
//     advanced from that minute to the end of p.
// The period's weather rows and the coefficient tables are read from LDS.
// Advancing a cell through a period costs one FBP evaluation; axes that
// reach their neighbour inside p offer that minute with atomicMin on the
// neighbour's 32-bit label, the rest become a continuation for p+1.
// Improved cells go to the period's work queue (LDS, spilling to the slot's
// global list): each wave reserves a range with one LDS atomic, writes its
// entries and commits the range in reservation order; waves take committed
// chunks of up to 64 entries as soon as they are free, so no wave waits for
// the others between hops.  The period ends when no wave holds a chunk and
// every reserved entry has been taken.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "device.h"
#include "kernels.h"
#include "types.h"

namespace c2f {

constexpr int32_t kNever = 0x7FFFFFFF;

__device__ __forceinline__ uint32_t load_label(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int wave_rank(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Value of x in lane `lane` (wave-uniform) without a trip through LDS.
__device__ __forceinline__ int lane_value(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }

// One LDS atomic per wave reserves slots for the appending lanes.
__device__ __forceinline__ int wave_reserve(bool pred, int* counter, uint64_t& m) {
    m = __ballot(pred);
    if (m == 0) return 0;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (__lane_id() == leader) base = atomicAdd(counter, (int)__popcll(m));
    return lane_value(base, leader) + wave_rank(m);
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


// ceil(r / q) for 0 < q < r < 2^16.  The float quotient x = r rcp(q) (rcp
// within one ulp) differs from r / q by less than (r / q) 2^-22, which is
// below 1 / q because r < 2^22.  With r / q = k + f: for f = 0, x lies in
// (k - 1, k + 1) and truncates to k - 1 or k; for f >= 1 / q, x lies in
// (k, k + 1) and truncates to k.  One exact 24-bit product then takes the
// truncation up to ceil(r / q) where it is one short.
__device__ __forceinline__ int32_t ceil_div_small(int32_t r, int32_t q) {
    uint32_t t = (uint32_t)((float)r * __builtin_amdgcn_rcpf((float)q));
    t += __umul24(t, (uint32_t)q) < (uint32_t)r;
    return (int32_t)t;
}

// Advance cell c (label lab) through period p from minute m0 to e.  nbv[k]
// is the label of neighbour k read at the start of the pass; rem[k] holds
// the metres left on axis k (0 = done).  On return cand[k] is the
// minute the fire reaches neighbour k inside p (or kNever) and rem[] the
// metres left at the end of p for axes still worth following.  An axis is
// dropped once its neighbour already holds a label no later candidate can
// beat, or is pending (its ignition minute is then already determined).
template <typename R>
__device__ __forceinline__ int advance(const RateCtx<R>& X, const CellRec& rec, uint32_t c, int p, int32_t m0,
                                       int32_t e, const uint32_t* nbv, uint32_t tag, int32_t* rem, int32_t* cand) {
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
        const bool faint = axis_q<R>(X, rec, c, (uint32_t)p, q);
        evals = 1;
        if (faint) {
            // burn-out (A5 (iv)): the head fire intensity is below the threshold
#pragma unroll
            for (int k = 0; k < 8; ++k) rem[k] = 0;
            return evals;
        }
        if (X.burnout > 0.f) {
            // burn-out (A5 (i)): every rate toward a burnable neighbour is
            // below delta, so the cell spreads no further
            int32_t qmax = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if ((nb >> k) & 1u) qmax = max(qmax, q[k]);
            if ((double)qmax < (double)X.burnout) {
#pragma unroll
                for (int k = 0; k < 8; ++k) rem[k] = 0;
                return evals;
            }
        }
        // minutes left in p; metres left per axis are below 2^16 (at most
        // the diagonal of a 20 km cell), so when q < r and n < r every
        // product below fits in 32 bits
        const int32_t n = e - m0 + 1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (!((live >> k) & 1u)) continue;
            const int32_t qk = q[k], r = rem[k];
            bool reach = false;
            int32_t step = 0;
            if (qk > 0) {
                if (qk >= r || n >= r) {
                    reach = true;
                } else {
                    // qk < r < 2^16 and n < r: a 24-bit product
                    step = (int32_t)__umul24((uint32_t)qk, (uint32_t)n);
                    reach = step >= r;
                }
            }
            if (reach) {
                cand[k] = m0 + (qk >= r ? 1 : ceil_div_small(r, qk)) - 1;
                rem[k] = 0;
            } else {
                rem[k] = r - step;
                if ((settled >> k) & 1u) rem[k] = 0;   // nothing after p can beat it
            }
        }
    }
    return evals;
}

// At least 2 waves per SIMD (<= 256 VGPRs).  A tighter bound (4 waves,
// 128 VGPRs) doubles the resident replications but spills several hundred
// bytes per lane to scratch in every pass, and measured slower; a 768-thread
// group needs 3 waves per SIMD (168 VGPRs) and a 1024-thread one 4 (128).
template <typename R, int BLOCK>
__global__ __launch_bounds__(BLOCK, 2) void propagate_kernel(const Job* __restrict__ jobs, int n_jobs,
                                                          int total_items, Slots slots,
                                                          RunCounters* __restrict__ rc) {
    constexpr int LCAP = BLOCK <= 64 ? 512 : (BLOCK <= 128 ? 1024 : (BLOCK <= 256 ? 2048 : 4096));
    constexpr int LQ = 2 * LCAP;   // LDS part of the period queue
    __shared__ uint2 s_Q[LQ];
    __shared__ int s_res, s_commit;   // queue entries reserved, committed (in order)
    // queue entries taken (high 32 bits) and waves holding a chunk (low 32),
    // one word so that taking a chunk and becoming a holder is one step
    __shared__ unsigned long long s_hb;
    __shared__ int s_nC[2], s_nP[2];
    __shared__ int s_item, s_flag;
    __shared__ uint32_t s_tag;
    __shared__ int s_scen, s_ign;
    // Decisions that steer every wave through the same barriers.  Each is
    // written by thread 0 only between two barriers and read by all
    // threads after the second, so no wave can read a value meant for a
    // later step: s_refill (the slot's plane needs refilling) and s_stop
    // (leave the period loop after this period).
    __shared__ int s_refill, s_stop;
    __shared__ unsigned long long s_cnt[kNumCounters];
    __shared__ CoefR<R> s_coef[kNumFuels];
    __shared__ CoefR<double> s_coef64[kNumFuels];
    __shared__ CoefR<float> s_coef32[kNumFuels];
    // the weather rows of the period being propagated (FP64, and FP32 where
    // the context evaluates in FP32 or tries FP32 first), staged at the
    // start of each period so that every evaluation reads them from LDS
    __shared__ double s_row64[kRowLen];
    __shared__ float s_row32[kRowLen];
    // the landscape's critical surface intensities, per fuel
    __shared__ double s_csi64[kNumFuels];
    __shared__ float s_csi32[kNumFuels];

    const int tid = threadIdx.x;
    const int slot = blockIdx.x;
    __builtin_amdgcn_s_setprio(1);
    if (tid < kNumFuels) {
        s_coef[tid] = coef_table<R>()[tid];
        s_coef64[tid] = coef_table<double>()[tid];
        s_coef32[tid] = coef_table<float>()[tid];
    }
    uint32_t* __restrict__ plane = slots.planes + (size_t)slot * (size_t)slots.plane_cells;
    const int64_t stride = slots.list_cap;   // entries allocated per list
    const int64_t cap = slots.list_limit;    // entries used per list (<= stride)
    uint8_t* lb = slots.lists + (size_t)slot * (size_t)stride * (size_t)kSlotListBytesPerEntry;
    uint2* const gQ = (uint2*)lb;        // global part of the period queue: 2 x cap entries
    Cont* const gC[2] = {(Cont*)(lb + 16 * stride), (Cont*)(lb + 16 * stride) + stride};
    uint32_t* const gP[2] = {(uint32_t*)(lb + 64 * stride), (uint32_t*)(lb + 64 * stride) + stride};

    for (int taken = 0;; ++taken) {
        // With deferred dense outputs (item_slot set) a slot's plane must
        // still hold its item's labels when the launch ends, so a group runs
        // at most one item; the launch then has a group for every item.
        if (slots.item_slot && taken > 0) break;
        if (tid == 0) {
            int it = atomicAdd(&rc->next_item, 1);
            if (__hip_atomic_load(&rc->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) it = total_items;
            else if (slots.order && it < total_items) it = slots.order[it];
            s_item = it;
        }
        __syncthreads();
        // values every thread reads from LDS after a barrier are the same in
        // every lane: readfirstlane tells the compiler so, which keeps the
        // job record and everything derived from it in scalar registers
        const int item = __builtin_amdgcn_readfirstlane(s_item);
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
        const int cols = job.cols;
        const int rows = job.rows;
        const int P = job.period_min;
        const CellRec* __restrict__ cells = job.cells;
        const bool use_thr = job.threshold > 0.0f;
        const R thr = (R)job.threshold;
        const int32_t D[8] = {job.d_orth, job.d_diag, job.d_orth, job.d_diag,
                              job.d_orth, job.d_diag, job.d_orth, job.d_diag};
        const int32_t off[8] = {1, 1 - cols, -cols, -cols - 1, -1, cols - 1, cols, cols + 1};
        const uint32_t last_cell = (uint32_t)((int64_t)rows * cols - 1);

        // ------------------------------------------- replication set-up
        if (tid < kNumFuels) {
            s_csi64[tid] = job.land->csi64[tid];
            s_csi32[tid] = job.land->csi32[tid];
        }
        if (tid == 0) {
            const uint32_t prev = slots.tags[slot];
            s_refill = prev <= 1u;   // tags exhausted: refill this slot's plane
            s_tag = prev <= 1u ? kTagFresh : prev;
            s_res = s_commit = 0;
            s_hb = 0ull;
            s_nC[0] = s_nC[1] = s_nP[0] = s_nP[1] = 0;
            s_flag = 0;
            s_stop = 0;
            for (int k = 0; k < kNumCounters; ++k) s_cnt[k] = 0;
            int scen, ign;
            rep_draws(job, rep, scen, ign);
            s_scen = scen;
            s_ign = ign;
        }
        __syncthreads();
        if (s_refill) {
            for (size_t i = tid; i < (size_t)slots.plane_cells; i += BLOCK) plane[i] = kPlaneFill;
            __syncthreads();
        }
        if (tid == 0) {
            const uint32_t tag = s_tag - 1u;
            s_tag = tag;
            slots.tags[slot] = tag;
            const int ign = s_ign;
            if (job.ign_mode != 4 && ign >= 0 && rec_fuel(cells[ign].info) != 0) {
                // the ignition takes the last minute before its period
                const uint32_t v = (tag << kMinuteBits) | (uint32_t)(job.ign_period * P);
                plane[ign] = v;
                s_Q[0] = make_uint2((uint32_t)ign, v);
                s_res = s_commit = 1;
                s_cnt[kCntIgnitions] = 1;
                if (job.count) atomicAdd(&job.count[ign], 1u);
            }
        }
        __syncthreads();
        const uint32_t tag = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_tag);
        const int scen_r = __builtin_amdgcn_readfirstlane(s_scen);
        const uint32_t pendv = (tag << kMinuteBits) | kPendingMinute;
        RateCtx<R> X;
        X.coef = s_coef;
        X.coef64 = s_coef64;
        X.L = land_consts<R>(job.land);
        X.L64 = land_consts<double>(job.land);
        if constexpr (sizeof(R) == 8) X.L.csi = (const R*)s_csi64;
        else X.L.csi = (const R*)s_csi32;
        X.L64.csi = s_csi64;
        const size_t so = (size_t)scen_r * job.n_wp * kRowLen;
        const double* const g_rows64 = job.table64 + so;
        const float* const g_rows32 =
            sizeof(R) == 4 ? (const float*)job.table + so : (job.table32 ? job.table32 + so : nullptr);
        if constexpr (sizeof(R) == 8) X.rows = (const R*)s_row64;
        else X.rows = (const R*)s_row32;
        X.rows64 = s_row64;
        X.row_stride = 0;
        X.coef32 = s_coef32;
        X.L32 = land_consts<float>(job.land);
        X.L32.csi = s_csi32;
        X.rows32 = g_rows32 ? s_row32 : nullptr;
        X.seed = job.seed;
        X.sigma = (R)job.sigma;
        X.rounding = job.rounding;
        X.rep = rep;
        X.burnout = job.burnout;
        X.hfi_min = job.hfi_min;

        uint32_t c_entries = 0, c_conts = 0, c_evals = 0, c_cand = 0, c_impr = 0, c_ign = 0, c_rounds = 0;
        int max_list = 0;
        int cc = 0, pc = 0;   // which buffer of each list pair is current
        const int64_t qcap = (int64_t)LQ + 2 * cap;   // queue entries per period

        // Append one entry per lane where `pred` holds: one reservation per
        // wave, entries written, then the range committed in reservation
        // order (earlier reservations never wait on later ones).  Called in
        // wave-uniform control flow.
        auto q_commit = [&](int wbase, int wtot) __attribute__((always_inline)) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (__lane_id() == 0) {
                while (__hip_atomic_load(&s_commit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != wbase)
                    __builtin_amdgcn_s_sleep(1);
                __hip_atomic_store(&s_commit, wbase + wtot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        };
        auto q_put = [&](int idx, uint2 val) __attribute__((always_inline)) {
            if (idx < LQ) s_Q[idx] = val;
            else if ((int64_t)(idx - LQ) < 2 * cap) gQ[idx - LQ] = val;
            else s_flag = 1;
        };
        auto q_append1 = [&](bool pred, uint2 val) __attribute__((always_inline)) {
            const uint64_t m = __ballot(pred);
            if (m == 0) return;
            int wbase = 0;
            if (__lane_id() == 0) wbase = atomicAdd(&s_res, (int)__popcll(m));
            wbase = lane_value(wbase, 0);
            if (pred) q_put(wbase + wave_rank(m), val);
            q_commit(wbase, (int)__popcll(m));
        };

        // the list's entries are sorted by period and the loop starts at the
        // earliest, so the entries of period p are those with period p, and
        // none is still to come after the last entry's period: both follow
        // from p alone, which every thread knows
        const int last_seed_period = job.n_seeds > 0 ? job.seeds[job.n_seeds - 1].y : -1;
        for (int p = job.ign_period; p < job.n_periods; ++p) {
            // list ignitions of period p take minute p P, inside or outside
            // the burning window, on cells with fuel that have not burned
            // (a pending cell included).  Lit by one thread between periods,
            // when no other thread touches the plane or the queue; an
            // improved label joins the queue like the set-up ignition.
            if (p <= last_seed_period && seeds_at(job, p)) {
                if (tid == 0) {
                    for (int k = 0; k < job.n_seeds; ++k) {
                        if (job.seeds[k].y != p) continue;
                        const uint32_t c = (uint32_t)job.seeds[k].x;
                        if (rec_fuel(cells[c].info) == 0) continue;
                        const uint32_t v = (tag << kMinuteBits) | (uint32_t)(job.seeds[k].y * P);
                        const uint32_t old = atomicMin(&plane[c], v);
                        if (v < old) {
                            if ((old >> kMinuteBits) != tag || (old & kMinuteMask) == kPendingMinute) {
                                ++c_ign;
                                if (job.count) atomicAdd(&job.count[c], 1u);
                            }
                            q_put(s_res, make_uint2(c, v));
                            s_commit = ++s_res;
                        }
                    }
                }
                __syncthreads();
            }
            // outside the daily burning window nothing spreads or ignites:
            // the continuations and pending cells wait, unchanged
            if (!burning_period(job, p)) continue;
            // every wave has left the previous period (its end barriers)
            for (int i = tid; i < kRowLen; i += BLOCK) {
                s_row64[i] = g_rows64[(size_t)p * kRowLen + i];
                if (g_rows32) s_row32[i] = g_rows32[(size_t)p * kRowLen + i];
            }
            __syncthreads();
            const int32_t s = p * P + 1;   // first minute of period p
            const int32_t e = (p + 1) * P; // last minute of period p

            // Each wave counts as a holder of the queue until it has done its
            // share of the pending cells and continuations below, so that no
            // wave finds the queue drained while another may still append to
            // it.  The waves then join the queue without a barrier: a wave
            // done early takes entries while others still advance
            // continuations (the labels are a least fixed point, whatever
            // the order).
            if (__lane_id() == 0) atomicAdd(&s_hb, 1ull);
            // Pending cells ignite at the start of p if their rate now passes;
            // the new labels join this period's queue.
            {
                const int nP = (int)min((int64_t)s_nP[pc], cap);
                for (int base = 0; base < nP; base += BLOCK) {
                    const int i = base + tid;
                    bool act = i < nP;
                    uint32_t j = 0;
                    if (act) {
                        j = gP[pc][i];
                        act = load_label(&plane[j]) == pendv;
                    }
                    bool ok = false;
                    if (act) {
                        const CellRec rj = cells[j];
                        ++c_evals;
                        ok = head_rate<R>(X, rj, j, (uint32_t)p) > thr;
                    }
                    bool improved = false, first = false;
                    const uint32_t v = (tag << kMinuteBits) | (uint32_t)s;
                    if (ok) {
                        const uint32_t old = atomicMin(&plane[j], v);
                        improved = v < old;
                        first = improved && ((old >> kMinuteBits) != tag || (old & kMinuteMask) == kPendingMinute);
                        if (first && job.count) atomicAdd(&job.count[j], 1u);
                    }
                    c_impr += improved;
                    c_ign += first;
                    q_append1(improved, make_uint2(j, v));
                    append_g(act && !ok, j, gP[pc ^ 1], cap, &s_nP[pc ^ 1], &s_flag);
                }
            }
            // Advance one entry per lane: the continuations of p-1 from the
            // start of p (conts), or a cell whose arrival improved inside p
            // from that minute.  Improvements are appended to the queue, axes
            // still travelling at the end of p to the next continuation list.
            auto process = [&](bool act, uint32_t c, uint32_t lab, int32_t* rem, bool conts) __attribute__((always_inline)) {
                int32_t cand[8];
                uint32_t nbv[8];
                CellRec rec;
                rec.info = 0;
                if (act) {
                    // issue every load of the entry at once: own label,
                    // cell record and the labels of the 8 neighbours.  A
                    // neighbour outside the grid is read at an index clamped
                    // into the plane (an index below 0 wraps to a large
                    // unsigned value and clamps too) and never used: the
                    // record's neighbour mask (in-grid burnable cells)
                    // excludes its axis.  Grids hold fewer than 2^31 cells.
                    const uint32_t own = load_label(&plane[c]);
                    rec = cells[c];
#pragma unroll
                    for (int k = 0; k < 8; ++k) nbv[k] = plane[min(c + (uint32_t)off[k], last_cell)];
                    act = own == lab;
                }
                bool keep = false;
                if (act) {
                    // a cell lit before p (an ignition waiting out the hours
                    // outside the burning window) advances from p's start
                    const int32_t m0 = conts ? s : max((int32_t)(lab & kMinuteMask) + 1, s);
                    c_evals += advance<R>(X, rec, c, p, m0, e, nbv, tag, rem, cand);
                    keep = (rem[0] | rem[1] | rem[2] | rem[3] | rem[4] | rem[5] | rem[6] | rem[7]) != 0;
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        cand[k] = kNever;
                        rem[k] = 0;
                    }
                }
                // offer the candidates: atomicMin of real labels, or a
                // pending mark where the neighbour's rate is below the
                // threshold.  All atomics are issued before any result is
                // used so that their latencies overlap.
                uint32_t hasm = 0, pendm = 0, impr = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) hasm |= (act && cand[k] != kNever) ? (1u << k) : 0u;
                if (use_thr) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        if (!((hasm >> k) & 1u)) continue;
                        const uint32_t j = (uint32_t)((int64_t)c + off[k]);
                        const CellRec rj = cells[j];
                        ++c_evals;
                        if (!(head_rate<R>(X, rj, j, (uint32_t)p) > thr)) pendm |= 1u << k;
                    }
                }
                uint32_t old[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    old[k] = 0u;
                    if ((hasm >> k) & 1u) {
                        const uint32_t v = ((pendm >> k) & 1u) ? pendv : (tag << kMinuteBits) | (uint32_t)cand[k];
                        old[k] = atomicMin(&plane[(int64_t)c + off[k]], v);
                    }
                }
                uint32_t newpend = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (!((hasm >> k) & 1u)) continue;
                    if ((pendm >> k) & 1u) {
                        if (old[k] > pendv) newpend |= 1u << k;
                        continue;
                    }
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
                // append the wave's improved neighbours axis by axis: one
                // ballot per axis gives each lane its place in the range
                c_impr += __popc(impr);
                uint64_t am[8];
                int wtot = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    am[k] = __ballot((impr >> k) & 1u);
                    wtot += (int)__popcll(am[k]);
                }
                if (wtot > 0) {
                    int wbase = 0;
                    if (__lane_id() == 0) wbase = atomicAdd(&s_res, wtot);
                    int idx = lane_value(wbase, 0);
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        if ((impr >> k) & 1u)
                            q_put(idx + wave_rank(am[k]),
                                  make_uint2((uint32_t)((int64_t)c + off[k]), (tag << kMinuteBits) | (uint32_t)cand[k]));
                        idx += (int)__popcll(am[k]);
                    }
                    q_commit(lane_value(wbase, 0), wtot);
                }
                if (use_thr) {
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        append_g(((newpend >> k) & 1u) != 0u, (uint32_t)((int64_t)c + off[k]), gP[pc ^ 1], cap,
                                 &s_nP[pc ^ 1], &s_flag);
                }
                // axes still travelling at the end of p continue in p+1
                Cont ct;
                ct.c = c;
                ct.label = lab;
#pragma unroll
                for (int h = 0; h < 4; ++h) ct.rem[h] = (uint32_t)rem[2 * h] | ((uint32_t)rem[2 * h + 1] << 16);
                append_g(keep, ct, gC[cc ^ 1], cap, &s_nC[cc ^ 1], &s_flag);
            };

            // Continuations of p-1, advanced from the start of p, last
            // listed first: the cells listed last were lit latest in p-1, at
            // the front of the fire, and tend to start the longest chains of
            // p, which then reach the queue in the first rounds.  Labels are
            // a least fixed point whatever the order.
            {
                const int n = (int)min((int64_t)s_nC[cc], cap);
                if (n > max_list) max_list = n;
                for (int base = 0; base < n; base += BLOCK) {
                    const int i = base + tid;
                    const bool act = i < n;
                    uint32_t c = 0, lab = 0;
                    int32_t rem[8];
                    if (act) {
                        const Cont ct = gC[cc][n - 1 - i];
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
            if (__lane_id() == 0) atomicAdd(&s_hb, ~0ull);   // no longer a holder

            // label correcting over the period's queue.  A wave waiting for
            // entries drops to the lowest issue priority, so that its polling
            // takes no issue slots from the waves working on the chain.
            for (;;) {
                int base = 0, cnt = 0;
                bool done = false;
                __builtin_amdgcn_s_setprio(0);
                if (__lane_id() == 0) {
                    for (;;) {
                        if (__hip_atomic_load(&s_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                            done = true;
                            break;
                        }
                        const unsigned long long hb =
                            __hip_atomic_load(&s_hb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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
                        // finished when no wave holds a chunk (so none can
                        // append) and every reserved entry has been taken
                        const int rs = __hip_atomic_load(&s_res, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        if (holders == 0 && h == cm && cm == rs) {
                            done = true;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                base = lane_value(base, 0);
                cnt = lane_value(cnt, 0);
                done = lane_value((int)done, 0) != 0;
                __builtin_amdgcn_s_setprio(1);
                if (done) break;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                ++c_rounds;
                const int i = base + __lane_id();
                bool act = __lane_id() < cnt && (int64_t)i < qcap;
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
            {
                const int n = s_res;
                if (n > max_list) max_list = n;
            }
            // ------------------------------------------------- period end
            // Thread 0 decides whether to stop between the two barriers: a
            // list overflowed, or the fire is out (no continuation and no
            // pending cell for p+1) and no listed ignition is still to
            // come.  Reading s_flag or the list lengths after the second
            // barrier could see values a faster wave already wrote in p+1.
            __syncthreads();
            if (tid == 0) {
                s_stop = s_flag || (s_nC[cc ^ 1] == 0 && s_nP[pc ^ 1] == 0 && last_seed_period <= p);
                s_nC[cc] = 0;
                s_nP[pc] = 0;
                s_res = s_commit = 0;
                s_hb = 0ull;
            }
            cc ^= 1;
            pc ^= 1;
            __syncthreads();
            if (s_stop) break;
        }
        if (s_flag && tid == 0) atomicOr(&rc->overflow, 1);

        // per-replication counters and outputs
        atomicAdd(&s_cnt[kCntIgnitions], (unsigned long long)c_ign);
        atomicAdd(&s_cnt[kCntEntries], (unsigned long long)c_entries);
        atomicAdd(&s_cnt[kCntConts], (unsigned long long)c_conts);
        atomicAdd(&s_cnt[kCntEvals], (unsigned long long)c_evals);
        atomicAdd(&s_cnt[kCntCandidates], (unsigned long long)c_cand);
        atomicAdd(&s_cnt[kCntImprovements], (unsigned long long)c_impr);
        if (__lane_id() == 0) atomicAdd(&s_cnt[kCntRounds], (unsigned long long)c_rounds);   // chunks, per wave
        atomicMax(&s_cnt[kCntMaxList], (unsigned long long)max_list);
        if (slots.item_slot) {
            if (tid == 0) slots.item_slot[item] = make_int2(slot, (int)tag);
        } else if (job.scar || job.arr_minute || job.arr_period) {
            __syncthreads();
            const size_t n = (size_t)job.rows * cols;
            const size_t o = (size_t)lr * n;
            for (size_t i = tid; i < n; i += BLOCK) {
                const uint32_t v = load_label(&plane[i]);
                const bool on = (v >> kMinuteBits) == tag && (v & kMinuteMask) != kPendingMinute;
                const int32_t t = on ? (int32_t)(v & kMinuteMask) : -1;
                if (job.scar) job.scar[o + i] = (uint8_t)on;
                if (job.arr_minute) job.arr_minute[o + i] = t;
                if (job.arr_period) job.arr_period[o + i] = !on ? -1 : (t == 0 ? 0 : (t - 1) / P);
            }
        }
        __syncthreads();
        if (tid == 0) {
            if (job.burned) job.burned[lr] = (int64_t)s_cnt[kCntIgnitions];
            if (job.ign_out) job.ign_out[lr] = s_ign;
            if (job.scen_out) job.scen_out[lr] = s_scen;
            for (int k = 0; k < kCntMaxList; ++k) atomicAdd(&rc->c[k], s_cnt[k]);
            atomicMax(&rc->c[kCntMaxList], s_cnt[kCntMaxList]);
        }
        __syncthreads();
    }
}

// Dense per-replication outputs from the final arrival planes, one thread
// per (item, cell): used when every item of the launch kept its own slot.
__global__ __launch_bounds__(256) void dense_outputs_kernel(const Job* __restrict__ jobs, int n_jobs,
                                                            int total_items, int n_slots, Slots slots,
                                                            const RunCounters* __restrict__ rc) {
    const int item = blockIdx.y;
    if (item >= total_items || rc->overflow) return;   // an overflowed launch is repeated
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].item_base <= item) lo = mid;
        else hi = mid - 1;
    }
    const Job& job = jobs[lo];
    if (!(job.scar || job.arr_minute || job.arr_period)) return;
    const int2 st = slots.item_slot[item];
    if (st.x < 0 || st.x >= n_slots) return;   // item not run (cleared to -1 before the launch)
    const uint32_t tag = (uint32_t)st.y;
    const uint32_t* __restrict__ plane = slots.planes + (size_t)st.x * (size_t)slots.plane_cells;
    const size_t n = (size_t)job.rows * (size_t)job.cols;
    const size_t o = (size_t)(item - job.item_base) * n;
    const int P = job.period_min;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t v = plane[i];
        const bool on = (v >> kMinuteBits) == tag && (v & kMinuteMask) != kPendingMinute;
        const int32_t t = on ? (int32_t)(v & kMinuteMask) : -1;
        if (job.scar) job.scar[o + i] = (uint8_t)on;
        if (job.arr_minute) job.arr_minute[o + i] = t;
        if (job.arr_period) job.arr_period[o + i] = !on ? -1 : (t == 0 ? 0 : (t - 1) / P);
    }
}

hipError_t launch_dense_outputs(const Job* jobs, int n_jobs, int total, int n_slots, int64_t max_cells,
                                const Slots& slots, const RunCounters* rc, hipStream_t s) {
    if (total <= 0 || total > 65535 || !slots.item_slot) return hipErrorInvalidValue;
    const int64_t want = (max_cells + 255) / 256;
    const int gx = (int)std::max<int64_t>(1, std::min<int64_t>(want, 4096 / std::min(total, 16)));
    hipLaunchKernelGGL(dense_outputs_kernel, dim3(gx, total), dim3(256), 0, s, jobs, n_jobs, total, n_slots, slots,
                       rc);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_prop_t(int block, int grid, const Job* jobs, int n_jobs, int total, const Slots& sl,
                                RunCounters* rc, hipStream_t s) {
    switch (block) {
        case 64: hipLaunchKernelGGL((propagate_kernel<R, 64>), dim3(grid), dim3(64), 0, s, jobs, n_jobs, total, sl, rc); break;
        case 128: hipLaunchKernelGGL((propagate_kernel<R, 128>), dim3(grid), dim3(128), 0, s, jobs, n_jobs, total, sl, rc); break;
        case 256: hipLaunchKernelGGL((propagate_kernel<R, 256>), dim3(grid), dim3(256), 0, s, jobs, n_jobs, total, sl, rc); break;
        case 512: hipLaunchKernelGGL((propagate_kernel<R, 512>), dim3(grid), dim3(512), 0, s, jobs, n_jobs, total, sl, rc); break;
        case 768: hipLaunchKernelGGL((propagate_kernel<R, 768>), dim3(grid), dim3(768), 0, s, jobs, n_jobs, total, sl, rc); break;
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
        case 768: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, propagate_kernel<R, 768>, 768, 0); break;
        case 1024: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, propagate_kernel<R, 1024>, 1024, 0); break;
        default: break;
    }
    return (e == hipSuccess) ? nb : 0;
}

int propagate_blocks_per_cu(int precision, int block) {
    return precision == 1 ? occ_t<float>(block) : occ_t<double>(block);
}

}  // namespace c2f
