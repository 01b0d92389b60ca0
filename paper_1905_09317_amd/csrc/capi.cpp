// libc2f host runtime: device memory, streams, work slots, relaunch on
// work-list overflow, batching of requests into one launch, hipGraph replay,
// autotuning, and the asynchronous serving queue.  Implements include/c2f.h.

#include "../../include/c2f.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fuel_table.h"
#include "kernels.h"
#include "types.h"

using namespace c2f;

namespace {

struct Landscape {
    int32_t rows = 0, cols = 0, cell_m = 0;
    float pc = 50.f, curing = 80.f;
    uint8_t* fuel = nullptr;
    CellRec* cells = nullptr;
    int32_t* burnable = nullptr;
    LandDev* land = nullptr;
    size_t bytes = 0;
    int64_t ncells() const { return (int64_t)rows * cols; }
};

struct Weather {
    int32_t n_scen = 0, n_periods = 0, period_min = 0;
    float* rows = nullptr;
    double* t64 = nullptr;
    float* t32 = nullptr;
    size_t bytes = 0;
};

struct TuneKey {
    int64_t cells;
    int32_t reps, precision;
    bool operator<(const TuneKey& o) const {
        if (cells != o.cells) return cells < o.cells;
        if (reps != o.reps) return reps < o.reps;
        return precision < o.precision;
    }
};

struct TuneVal {
    int32_t block;
    int64_t list_cap;
};

// Host-side view of a request's outputs and where the kernel writes them.
struct OutPlan {
    c2f_outputs user{};
    // device destinations (either user pointers or staging)
    uint8_t* scar = nullptr;
    int32_t* arr_period = nullptr;
    int32_t* arr_minute = nullptr;
    uint32_t* count = nullptr;
    int64_t* burned = nullptr;
    int32_t* ign = nullptr;
    int32_t* scen = nullptr;
};

struct Ticket;

}  // namespace

struct c2f_ctx {
    int device = 0;
    uint64_t budget = 0;
    int n_cu = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    std::string err;
    std::map<int32_t, Landscape> lands;
    std::map<int32_t, Weather> weathers;
    int32_t next_id = 1;
    size_t bytes_in_use = 0;

    // work slots
    uint32_t* planes = nullptr;
    int64_t plane_cells = 0;
    int32_t n_slots = 0;
    uint8_t* lists = nullptr;
    int64_t list_cap = 0;
    int32_t list_slots = 0;
    uint32_t* tags = nullptr;
    int32_t tag_slots = 0;

    RunCounters* rc = nullptr;
    RunCounters* rc_host = nullptr;   // pinned
    Job* d_jobs = nullptr;
    int32_t d_jobs_cap = 0;
    Job* h_jobs = nullptr;            // pinned
    int32_t h_jobs_cap = 0;

    void* staging = nullptr;
    size_t staging_bytes = 0;

    int32_t block_override = 0;
    int64_t cap_override = 0;
    std::map<TuneKey, TuneVal> tune;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    c2f_run_stats last{};

    // hipGraph of the last plain launch sequence
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<uint64_t> graph_key;
    bool graph_unavailable = false;   // capture refused once: launch eagerly

    std::mutex mu;   // serialises device work between API calls and the server thread

    // serving
    std::mutex smu;
    std::condition_variable scv;
    std::deque<std::shared_ptr<Ticket>> queue;
    std::map<uint64_t, std::shared_ptr<Ticket>> tickets;
    uint64_t next_ticket = 1;
    std::thread server;
    bool stopping = false;
    int32_t max_queue = 4096;
    int32_t max_batch_items = 1 << 16;
};

namespace {

struct Ticket {
    uint64_t id = 0;
    c2f_sim_params params{};
    c2f_outputs out{};
    bool done = false;
    c2f_status status = C2F_OK;
    std::string err;
    size_t footprint = 0;
};

// Drop any error left by an earlier runtime call whose status was ignored,
// so that launch checks (hipGetLastError) report only their own launch.
inline void clear_sticky_error() { (void)hipGetLastError(); }

c2f_status fail(c2f_ctx* ctx, c2f_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}

#define HIP_TRY(ctx, expr)                                                                         \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((ctx), C2F_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

c2f_status dev_alloc(c2f_ctx* ctx, void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (ctx->budget && ctx->bytes_in_use + bytes > ctx->budget)
        return fail(ctx, C2F_ENOMEM, "HBM budget exceeded: %zu in use + %zu requested > %llu", ctx->bytes_in_use,
                    bytes, (unsigned long long)ctx->budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(ctx, C2F_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    ctx->bytes_in_use += bytes;
    return C2F_OK;
}

void dev_free(c2f_ctx* ctx, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    if (bytes == 0) bytes = 16;
    ctx->bytes_in_use -= std::min(ctx->bytes_in_use, bytes);
}

int32_t axis_diag(int32_t cs) {
    // least integer D with D*D >= 2 cs^2
    const int64_t two = 2ll * cs * cs;
    int64_t d = (int64_t)std::sqrt((double)two);
    while (d * d < two) ++d;
    while ((d - 1) * (d - 1) >= two) --d;
    return (int32_t)d;
}

void drop_graph(c2f_ctx* ctx) {
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    clear_sticky_error();
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_key.clear();
}

// Make sure n slots of plane_cells labels and lists of `cap` entries exist.
c2f_status ensure_slots(c2f_ctx* ctx, int32_t n, int64_t cells, int64_t cap) {
    if (n > ctx->n_slots || cells > ctx->plane_cells) {
        drop_graph(ctx);
        dev_free(ctx, ctx->planes, (size_t)ctx->n_slots * ctx->plane_cells * 4);
        ctx->planes = nullptr;
        const int32_t ns = std::max(n, ctx->n_slots);
        const int64_t pc = std::max(cells, ctx->plane_cells);
        ctx->n_slots = 0;
        ctx->plane_cells = 0;
        c2f_status st = dev_alloc(ctx, (void**)&ctx->planes, (size_t)ns * pc * 4);
        if (st != C2F_OK) return st;
        ctx->n_slots = ns;
        ctx->plane_cells = pc;
        HIP_TRY(ctx, launch_fill_u32(ctx->planes, (size_t)ns * pc, kPlaneFill, ctx->stream));
        // every slot restarts from a freshly filled plane
        dev_free(ctx, ctx->tags, (size_t)ctx->tag_slots * 4);
        ctx->tags = nullptr;
        ctx->tag_slots = 0;
        st = dev_alloc(ctx, (void**)&ctx->tags, (size_t)ns * 4);
        if (st != C2F_OK) return st;
        ctx->tag_slots = ns;
        HIP_TRY(ctx, launch_fill_u32(ctx->tags, (size_t)ns, kTagFresh, ctx->stream));
    }
    if (n > ctx->list_slots || cap != ctx->list_cap) {
        drop_graph(ctx);
        dev_free(ctx, ctx->lists, (size_t)ctx->list_slots * ctx->list_cap * kSlotListBytesPerEntry);
        ctx->lists = nullptr;
        const int32_t ns = std::max(n, ctx->list_slots);
        ctx->list_slots = 0;
        ctx->list_cap = 0;
        c2f_status st = dev_alloc(ctx, (void**)&ctx->lists, (size_t)ns * cap * kSlotListBytesPerEntry);
        if (st != C2F_OK) return st;
        ctx->list_slots = ns;
        ctx->list_cap = cap;
    }
    return C2F_OK;
}

c2f_status ensure_jobs(c2f_ctx* ctx, int32_t n) {
    if (n > ctx->d_jobs_cap) {
        drop_graph(ctx);
        dev_free(ctx, ctx->d_jobs, (size_t)ctx->d_jobs_cap * sizeof(Job));
        ctx->d_jobs = nullptr;
        ctx->d_jobs_cap = 0;
        const int32_t cap = std::max(n, 64);
        c2f_status st = dev_alloc(ctx, (void**)&ctx->d_jobs, (size_t)cap * sizeof(Job));
        if (st != C2F_OK) return st;
        ctx->d_jobs_cap = cap;
    }
    if (n > ctx->h_jobs_cap) {
        if (ctx->h_jobs) (void)hipHostFree(ctx->h_jobs);
        ctx->h_jobs = nullptr;
        ctx->h_jobs_cap = 0;
        const int32_t cap = std::max(n, 64);
        HIP_TRY(ctx, hipHostMalloc((void**)&ctx->h_jobs, (size_t)cap * sizeof(Job), hipHostMallocDefault));
        ctx->h_jobs_cap = cap;
    }
    return C2F_OK;
}

c2f_status ensure_staging(c2f_ctx* ctx, size_t bytes) {
    if (bytes > ctx->staging_bytes) {
        drop_graph(ctx);
        dev_free(ctx, ctx->staging, ctx->staging_bytes);
        ctx->staging = nullptr;
        ctx->staging_bytes = 0;
        c2f_status st = dev_alloc(ctx, &ctx->staging, bytes);
        if (st != C2F_OK) return st;
        ctx->staging_bytes = bytes;
    }
    return C2F_OK;
}

c2f_status check_params(c2f_ctx* ctx, const c2f_sim_params* p, const Landscape** L, const Weather** W) {
    if (!p) return fail(ctx, C2F_EINVAL, "params is NULL");
    auto li = ctx->lands.find(p->landscape_id);
    if (li == ctx->lands.end()) return fail(ctx, C2F_ESTATE, "unknown landscape id %d", p->landscape_id);
    auto wi = ctx->weathers.find(p->weather_id);
    if (wi == ctx->weathers.end()) return fail(ctx, C2F_ESTATE, "unknown weather id %d", p->weather_id);
    const Landscape& l = li->second;
    const Weather& w = wi->second;
    if (p->reps <= 0) return fail(ctx, C2F_EINVAL, "reps must be >= 1 (got %d)", p->reps);
    if (p->rep_offset < 0 || (int64_t)p->rep_offset + p->reps > 0x7FFFFFFFll)
        return fail(ctx, C2F_EINVAL, "rep_offset out of range");
    if (p->n_periods <= 0 || p->n_periods > w.n_periods)
        return fail(ctx, C2F_EINVAL, "n_periods %d not in 1..%d (weather periods)", p->n_periods, w.n_periods);
    if ((int64_t)p->n_periods * w.period_min > kMaxMinutes)
        return fail(ctx, C2F_EINVAL, "run too long: %lld minutes > %d", (long long)p->n_periods * w.period_min,
                    kMaxMinutes);
    if (!(p->ros_sigma >= 0.f) || !std::isfinite(p->ros_sigma))
        return fail(ctx, C2F_EINVAL, "ros_sigma must be finite and >= 0");
    if (!std::isfinite(p->ros_threshold)) return fail(ctx, C2F_EINVAL, "ros_threshold must be finite");
    if (p->rounding != 0 && p->rounding != 1) return fail(ctx, C2F_EINVAL, "rounding must be 0 or 1");
    if (p->precision != 0 && p->precision != 1) return fail(ctx, C2F_EINVAL, "precision must be 0 or 1");
    if (p->ignition_mode < 0 || p->ignition_mode > 2) return fail(ctx, C2F_EINVAL, "ignition_mode must be 0..2");
    if (p->ignition_mode == 0 && (p->ignition_cell < 0 || p->ignition_cell >= l.ncells()))
        return fail(ctx, C2F_EINVAL, "ignition_cell %d outside the grid", p->ignition_cell);
    if (p->scenario_mode < 0 || p->scenario_mode > 1) return fail(ctx, C2F_EINVAL, "scenario_mode must be 0 or 1");
    if (p->scenario_mode == 0 && (p->scenario < 0 || p->scenario >= w.n_scen))
        return fail(ctx, C2F_EINVAL, "scenario %d not in 0..%d", p->scenario, w.n_scen - 1);
    *L = &l;
    *W = &w;
    return C2F_OK;
}

int64_t default_list_cap(int64_t cells, int32_t reps) {
    // Generous for single large fires, modest when many slots share HBM;
    // an overflow is detected and the run repeated with twice the capacity.
    int64_t cap = reps <= 64 ? (int64_t)1 << 20 : (int64_t)1 << 16;
    cap = std::min<int64_t>(cap, std::max<int64_t>(1024, 2 * cells));
    return cap;
}

struct LaunchPlan {
    int32_t block = 256;
    int32_t grid = 1;
    int64_t cap = 1024;
};

LaunchPlan plan_launch(c2f_ctx* ctx, int64_t cells, int32_t total_items, int32_t precision) {
    LaunchPlan lp;
    auto it = ctx->tune.find(TuneKey{cells, total_items, precision});
    if (it != ctx->tune.end()) {
        lp.block = it->second.block;
        lp.cap = it->second.list_cap;
    } else {
        lp.block = cells >= (1 << 22) && total_items <= 16 ? 1024 : 256;
        lp.cap = default_list_cap(cells, total_items);
    }
    if (ctx->block_override) lp.block = ctx->block_override;
    if (ctx->cap_override) lp.cap = ctx->cap_override;
    int per_cu = propagate_blocks_per_cu(precision, lp.block);
    if (per_cu < 1) per_cu = 1;
    lp.grid = std::max(1, std::min(total_items, per_cu * ctx->n_cu));
    return lp;
}

// One fused launch over all requests of one precision.  Relaunches with a
// larger list capacity if any work list overflowed.
c2f_status run_group(c2f_ctx* ctx, const std::vector<int>& idx, const std::vector<c2f_sim_params>& P,
                     const std::vector<const Landscape*>& Ls, const std::vector<const Weather*>& Ws,
                     std::vector<OutPlan>& plans, int32_t precision, bool use_graph) {
    if (idx.empty()) return C2F_OK;
    int64_t max_cells = 0;
    int32_t total = 0;
    for (int k : idx) {
        max_cells = std::max(max_cells, Ls[k]->ncells());
        total += P[k].reps;
    }
    LaunchPlan lp = plan_launch(ctx, max_cells, total, precision);
    c2f_status st = ensure_jobs(ctx, (int32_t)idx.size());
    if (st != C2F_OK) return st;

    for (;;) {
        st = ensure_slots(ctx, lp.grid, max_cells, lp.cap);
        if (st == C2F_ENOMEM && lp.grid > 1) {
            // fewer resident slots still computes the same result
            lp.grid = std::max(1, lp.grid / 2);
            continue;
        }
        if (st != C2F_OK) return st;

        int32_t item = 0;
        for (size_t q = 0; q < idx.size(); ++q) {
            const int k = idx[q];
            const c2f_sim_params& p = P[k];
            const Landscape& L = *Ls[k];
            const Weather& W = *Ws[k];
            const OutPlan& o = plans[k];
            Job j;
            memset(&j, 0, sizeof j);
            j.cells = L.cells;
            j.burnable = L.burnable;
            j.land = L.land;
            j.table = precision == 1 ? (const void*)W.t32 : (const void*)W.t64;
            j.table64 = W.t64;
            j.rows = L.rows;
            j.cols = L.cols;
            j.d_orth = L.cell_m;
            j.d_diag = axis_diag(L.cell_m);
            j.n_scen = W.n_scen;
            j.n_wp = W.n_periods;
            j.period_min = W.period_min;
            j.n_periods = p.n_periods;
            j.T = p.n_periods * W.period_min;
            j.reps = p.reps;
            j.rep_offset = p.rep_offset;
            j.item_base = item;
            j.rounding = p.rounding;
            j.ign_mode = p.ignition_mode;
            j.ign_cell = p.ignition_cell;
            j.scen_mode = p.scenario_mode;
            j.scen_fixed = p.scenario;
            j.sigma = p.ros_sigma;
            j.threshold = p.ros_threshold;
            j.seed = p.seed;
            j.scar = o.scar;
            j.arr_period = o.arr_period;
            j.arr_minute = o.arr_minute;
            j.count = o.count;
            j.burned = o.burned;
            j.ign_out = o.ign;
            j.scen_out = o.scen;
            ctx->h_jobs[q] = j;
            item += p.reps;
        }
        HIP_TRY(ctx, hipMemcpyAsync(ctx->d_jobs, ctx->h_jobs, idx.size() * sizeof(Job), hipMemcpyHostToDevice,
                                    ctx->stream));

        Slots sl{ctx->planes, ctx->plane_cells, ctx->lists, ctx->list_cap, ctx->tags};
        // key of the launch sequence for graph reuse
        std::vector<uint64_t> key = {(uint64_t)(uintptr_t)ctx->d_jobs, idx.size(), (uint64_t)total,
                                     (uint64_t)lp.block, (uint64_t)lp.grid, (uint64_t)precision,
                                     (uint64_t)(uintptr_t)ctx->planes, (uint64_t)(uintptr_t)ctx->lists,
                                     (uint64_t)ctx->list_cap, (uint64_t)ctx->plane_cells,
                                     (uint64_t)(uintptr_t)ctx->stream};
        for (int k : idx) {
            key.push_back((uint64_t)(uintptr_t)plans[k].count);
            key.push_back((uint64_t)Ls[k]->ncells());
        }
        // fills + propagation; the events bracket this sequence (they are
        // recorded outside any graph capture)
        auto enqueue = [&]() -> hipError_t {
            hipError_t e = launch_fill_u32((uint32_t*)ctx->rc, sizeof(RunCounters) / 4, 0u, ctx->stream);
            if (e != hipSuccess) return e;
            for (int k : idx) {
                if (plans[k].count) {
                    e = launch_fill_u32(plans[k].count, (size_t)Ls[k]->ncells(), 0u, ctx->stream);
                    if (e != hipSuccess) return e;
                }
            }
            return launch_propagate(precision, lp.block, lp.grid, ctx->d_jobs, (int)idx.size(), total, sl,
                                    ctx->rc, ctx->stream);
        };
        bool launched = false;
        if (use_graph && !ctx->graph_unavailable) {
            if (ctx->graph_exec == nullptr || ctx->graph_key != key) {
                drop_graph(ctx);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    hipError_t e1 = enqueue();
                    hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
                    e = (e1 != hipSuccess) ? e1 : e2;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    if (g) (void)hipGraphDestroy(g);
                    ctx->graph_exec = nullptr;
                    ctx->graph_unavailable = true;
                } else {
                    ctx->graph = g;
                    ctx->graph_key = key;
                }
            }
            if (ctx->graph_exec) {
                HIP_TRY(ctx, hipEventRecord(ctx->ev0, ctx->stream));
                HIP_TRY(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
                HIP_TRY(ctx, hipEventRecord(ctx->ev1, ctx->stream));
                launched = true;
            }
        }
        if (!launched) {
            HIP_TRY(ctx, hipEventRecord(ctx->ev0, ctx->stream));
            HIP_TRY(ctx, enqueue());
            HIP_TRY(ctx, hipEventRecord(ctx->ev1, ctx->stream));
        }
        HIP_TRY(ctx, hipMemcpyAsync(ctx->rc_host, ctx->rc, sizeof(RunCounters), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ctx->last.kernel_ms += ms;
        if (ctx->rc_host->overflow == 0) {
            ctx->last.entries += (int64_t)ctx->rc_host->c[kCntEntries];
            ctx->last.rate_evals += (int64_t)ctx->rc_host->c[kCntEvals];
            ctx->last.candidates += (int64_t)ctx->rc_host->c[kCntCandidates];
            ctx->last.improvements += (int64_t)ctx->rc_host->c[kCntImprovements];
            ctx->last.ignitions += (int64_t)ctx->rc_host->c[kCntIgnitions];
            ctx->last.rounds += (int64_t)ctx->rc_host->c[kCntRounds];
            ctx->last.continuations += (int64_t)ctx->rc_host->c[kCntConts];
            ctx->last.block_threads = lp.block;
            ctx->last.grid_blocks = lp.grid;
            ctx->last.list_capacity = lp.cap;
            return C2F_OK;
        }
        ++ctx->last.relaunches;
        const int64_t hard_max = std::min<int64_t>(std::max<int64_t>(4 * max_cells, 1 << 12) * 8, (int64_t)1 << 30);
        if (lp.cap >= hard_max) return fail(ctx, C2F_ECAPACITY, "work lists overflow at capacity %lld", (long long)lp.cap);
        lp.cap = std::min(hard_max, lp.cap * 4);
        // remember the larger capacity for requests of this shape
        ctx->tune[TuneKey{max_cells, total, precision}] = TuneVal{lp.block, lp.cap};
    }
}

c2f_status simulate_impl(c2f_ctx* ctx, int32_t n_jobs, const c2f_sim_params* params, const c2f_outputs* outs,
                         bool use_graph) {
    if (!ctx) return C2F_EINVAL;
    if (n_jobs <= 0 || !params || !outs) return fail(ctx, C2F_EINVAL, "need n_jobs >= 1 and params/out arrays");
    std::vector<c2f_sim_params> P(params, params + n_jobs);
    std::vector<const Landscape*> Ls(n_jobs);
    std::vector<const Weather*> Ws(n_jobs);
    int64_t total_items = 0;
    for (int k = 0; k < n_jobs; ++k) {
        c2f_status st = check_params(ctx, &P[k], &Ls[k], &Ws[k]);
        if (st != C2F_OK) return st;
        total_items += P[k].reps;
    }
    if (total_items > 0x3FFFFFFF) return fail(ctx, C2F_EINVAL, "too many replications in one call");

    // plan outputs: device pointers directly, host ones through staging
    std::vector<OutPlan> plans(n_jobs);
    size_t stage = 0;
    auto need = [&](bool want, size_t bytes) -> size_t {
        if (!want) return 0;
        const size_t off = stage;
        stage += (bytes + 255) & ~(size_t)255;
        return off + 1;   // +1 so that 0 means "none"
    };
    std::vector<std::array<size_t, 7>> offs(n_jobs);
    for (int k = 0; k < n_jobs; ++k) {
        const c2f_outputs& o = outs[k];
        plans[k].user = o;
        const size_t n = (size_t)Ls[k]->ncells(), r = (size_t)P[k].reps;
        if (o.on_device) {
            plans[k].scar = o.scar;
            plans[k].arr_period = o.arrival_period;
            plans[k].arr_minute = o.arrival_minute;
            plans[k].count = o.burn_count;
            plans[k].burned = o.burned_cells;
            plans[k].ign = o.ignition_cell;
            plans[k].scen = o.scenario;
        } else {
            offs[k] = {need(o.scar, r * n), need(o.arrival_period, r * n * 4), need(o.arrival_minute, r * n * 4),
                       need(o.burn_count, n * 4), need(o.burned_cells, r * 8), need(o.ignition_cell, r * 4),
                       need(o.scenario, r * 4)};
        }
    }
    c2f_status st = ensure_staging(ctx, stage);
    if (st != C2F_OK) return st;
    char* sb = (char*)ctx->staging;
    for (int k = 0; k < n_jobs; ++k) {
        if (outs[k].on_device) continue;
        auto at = [&](size_t off) -> void* { return off ? sb + off - 1 : nullptr; };
        plans[k].scar = (uint8_t*)at(offs[k][0]);
        plans[k].arr_period = (int32_t*)at(offs[k][1]);
        plans[k].arr_minute = (int32_t*)at(offs[k][2]);
        plans[k].count = (uint32_t*)at(offs[k][3]);
        plans[k].burned = (int64_t*)at(offs[k][4]);
        plans[k].ign = (int32_t*)at(offs[k][5]);
        plans[k].scen = (int32_t*)at(offs[k][6]);
    }

    memset(&ctx->last, 0, sizeof ctx->last);
    std::vector<int> g64, g32;
    for (int k = 0; k < n_jobs; ++k) (P[k].precision == 1 ? g32 : g64).push_back(k);
    if (!g64.empty() && !g32.empty()) use_graph = false;   // one cached graph per context
    st = run_group(ctx, g64, P, Ls, Ws, plans, 0, use_graph);
    if (st != C2F_OK) return st;
    st = run_group(ctx, g32, P, Ls, Ws, plans, 1, use_graph);
    if (st != C2F_OK) return st;

    // copy host outputs back
    for (int k = 0; k < n_jobs; ++k) {
        const c2f_outputs& o = outs[k];
        if (o.on_device) continue;
        const size_t n = (size_t)Ls[k]->ncells(), r = (size_t)P[k].reps;
        auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
            if (!dst) return hipSuccess;
            return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream);
        };
        HIP_TRY(ctx, cp(o.scar, plans[k].scar, r * n));
        HIP_TRY(ctx, cp(o.arrival_period, plans[k].arr_period, r * n * 4));
        HIP_TRY(ctx, cp(o.arrival_minute, plans[k].arr_minute, r * n * 4));
        HIP_TRY(ctx, cp(o.burn_count, plans[k].count, n * 4));
        HIP_TRY(ctx, cp(o.burned_cells, plans[k].burned, r * 8));
        HIP_TRY(ctx, cp(o.ignition_cell, plans[k].ign, r * 4));
        HIP_TRY(ctx, cp(o.scenario, plans[k].scen, r * 4));
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return C2F_OK;
}

size_t request_footprint(const c2f_ctx* ctx, const c2f_sim_params& p) {
    auto li = ctx->lands.find(p.landscape_id);
    if (li == ctx->lands.end()) return 0;
    const size_t n = (size_t)li->second.ncells();
    // staging of the outputs the serving path may return (counts + per-rep)
    return n * 4 + (size_t)p.reps * 24;
}

void server_loop(c2f_ctx* ctx);

}  // namespace

// ===================================================================== ABI

extern "C" {

c2f_status c2f_create(int32_t device, uint64_t hbm_budget_bytes, c2f_ctx** out) {
    if (!out) return C2F_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return C2F_EDEVICE;
    }
    if (device < 0 || device >= n) return C2F_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return C2F_EDEVICE;
    std::unique_ptr<c2f_ctx> ctx(new c2f_ctx());
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return C2F_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return C2F_EDEVICE;
    ctx->n_cu = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking) != hipSuccess) return C2F_EDEVICE;
    ctx->stream = ctx->own_stream;
    if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess) return C2F_EDEVICE;
    if (dev_alloc(ctx.get(), (void**)&ctx->rc, sizeof(RunCounters)) != C2F_OK) return C2F_ENOMEM;
    if (hipHostMalloc((void**)&ctx->rc_host, sizeof(RunCounters), hipHostMallocDefault) != hipSuccess)
        return C2F_EDEVICE;
    *out = ctx.release();
    return C2F_OK;
}

void c2f_destroy(c2f_ctx* ctx) {
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> lk(ctx->smu);
        ctx->stopping = true;
    }
    ctx->scv.notify_all();
    if (ctx->server.joinable()) ctx->server.join();
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
    for (auto& kv : ctx->lands) {
        (void)hipFree(kv.second.fuel);
        (void)hipFree(kv.second.cells);
        (void)hipFree(kv.second.burnable);
        (void)hipFree(kv.second.land);
    }
    for (auto& kv : ctx->weathers) {
        (void)hipFree(kv.second.rows);
        (void)hipFree(kv.second.t64);
        (void)hipFree(kv.second.t32);
    }
    (void)hipFree(ctx->planes);
    (void)hipFree(ctx->lists);
    (void)hipFree(ctx->tags);
    (void)hipFree(ctx->rc);
    (void)hipFree(ctx->d_jobs);
    (void)hipFree(ctx->staging);
    if (ctx->h_jobs) (void)hipHostFree(ctx->h_jobs);
    if (ctx->rc_host) (void)hipHostFree(ctx->rc_host);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    delete ctx;
}

const char* c2f_last_error(const c2f_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

c2f_status c2f_set_stream(c2f_ctx* ctx, void* hip_stream) {
    if (!ctx) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
    drop_graph(ctx);
    ctx->stream = hip_stream ? (hipStream_t)hip_stream : ctx->own_stream;
    return C2F_OK;
}

c2f_status c2f_load_landscape(c2f_ctx* ctx, int32_t rows, int32_t cols, int32_t cell_m, const uint8_t* fuel,
                              const int16_t* elev_m, float pc_pct, float curing_pct, int32_t* landscape_id) {
    if (!ctx) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
    ctx->err.clear();
    if (rows <= 0 || cols <= 0 || (int64_t)rows * cols > 0x7FFFFFFEll)
        return fail(ctx, C2F_EINVAL, "grid %d x %d out of range", rows, cols);
    if (cell_m < 1 || cell_m > 20000) return fail(ctx, C2F_EINVAL, "cell_m %d not in 1..20000", cell_m);
    if (!fuel || !landscape_id) return fail(ctx, C2F_EINVAL, "fuel and landscape_id must be non-NULL");
    if (!(pc_pct >= 0.f && pc_pct <= 100.f)) return fail(ctx, C2F_EINVAL, "pc_pct must be in 0..100");
    if (!(curing_pct > 0.f && curing_pct <= 100.f)) return fail(ctx, C2F_EINVAL, "curing_pct must be in (0, 100]");
    const int64_t n = (int64_t)rows * cols;
    for (int64_t i = 0; i < n; ++i)
        if (fuel[i] > 15) return fail(ctx, C2F_EINVAL, "fuel code %d at cell %lld > 15", fuel[i], (long long)i);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    Landscape L;
    L.rows = rows;
    L.cols = cols;
    L.cell_m = cell_m;
    L.pc = pc_pct;
    L.curing = curing_pct;
    int16_t* d_elev = nullptr;
    int32_t* d_tiles = nullptr;
    const int64_t n_tiles = tile_scratch_entries(n);
    c2f_status st = C2F_OK;
    auto cleanup = [&]() {
        dev_free(ctx, L.fuel, (size_t)n);
        dev_free(ctx, L.cells, (size_t)n * sizeof(CellRec));
        dev_free(ctx, L.burnable, (size_t)n * 4);
        dev_free(ctx, L.land, sizeof(LandDev));
        dev_free(ctx, d_elev, (size_t)n * 2);
        dev_free(ctx, d_tiles, (size_t)n_tiles * 4);
    };
    if ((st = dev_alloc(ctx, (void**)&L.fuel, (size_t)n)) != C2F_OK ||
        (st = dev_alloc(ctx, (void**)&L.cells, (size_t)n * sizeof(CellRec))) != C2F_OK ||
        (st = dev_alloc(ctx, (void**)&L.burnable, (size_t)n * 4)) != C2F_OK ||
        (st = dev_alloc(ctx, (void**)&L.land, sizeof(LandDev))) != C2F_OK ||
        (st = dev_alloc(ctx, (void**)&d_tiles, (size_t)n_tiles * 4)) != C2F_OK ||
        (elev_m && (st = dev_alloc(ctx, (void**)&d_elev, (size_t)n * 2)) != C2F_OK)) {
        cleanup();
        return st;
    }
    hipError_t e = hipMemcpyAsync(L.fuel, fuel, (size_t)n, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess && elev_m) e = hipMemcpyAsync(d_elev, elev_m, (size_t)n * 2, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_prepare_landscape(L.fuel, d_elev, rows, cols, cell_m, pc_pct, curing_pct, L.cells, L.burnable,
                                     d_tiles, L.land, ctx->stream);
    LandDev hl;
    if (e == hipSuccess) e = hipMemcpyAsync(&hl, L.land, sizeof hl, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dev_free(ctx, d_elev, (size_t)n * 2);
    d_elev = nullptr;
    dev_free(ctx, d_tiles, (size_t)n_tiles * 4);
    d_tiles = nullptr;
    if (e != hipSuccess) {
        cleanup();
        return fail(ctx, C2F_EDEVICE, "landscape preparation failed: %s", hipGetErrorString(e));
    }
    if (hl.grad_overflow) {
        cleanup();
        return fail(ctx, C2F_EINVAL, "elevation too steep: a Horn gradient numerator exceeds 32767");
    }
    L.bytes = (size_t)n * (1 + sizeof(CellRec) + 4) + sizeof(LandDev);
    const int32_t id = ctx->next_id++;
    ctx->lands[id] = L;
    *landscape_id = id;
    return C2F_OK;
}

c2f_status c2f_unload_landscape(c2f_ctx* ctx, int32_t landscape_id) {
    if (!ctx) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
    auto it = ctx->lands.find(landscape_id);
    if (it == ctx->lands.end()) return fail(ctx, C2F_ESTATE, "unknown landscape id %d", landscape_id);
    (void)hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
    Landscape& L = it->second;
    const size_t n = (size_t)L.ncells();
    dev_free(ctx, L.fuel, n);
    dev_free(ctx, L.cells, n * sizeof(CellRec));
    dev_free(ctx, L.burnable, n * 4);
    dev_free(ctx, L.land, sizeof(LandDev));
    ctx->lands.erase(it);
    return C2F_OK;
}

c2f_status c2f_set_weather(c2f_ctx* ctx, int32_t n_scen, int32_t n_periods, int32_t period_min,
                           const c2f_weather_row* rows, int32_t* weather_id) {
    if (!ctx) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
    ctx->err.clear();
    if (n_scen <= 0 || n_periods <= 0 || period_min <= 0 || !rows || !weather_id)
        return fail(ctx, C2F_EINVAL, "need n_scen, n_periods, period_min >= 1 and non-NULL rows/weather_id");
    if ((int64_t)n_scen * n_periods > (1 << 26)) return fail(ctx, C2F_EINVAL, "weather table too large");
    const int64_t nr = (int64_t)n_scen * n_periods;
    for (int64_t i = 0; i < nr; ++i) {
        const c2f_weather_row& w = rows[i];
        if (!(w.ffmc >= 0.f && w.ffmc <= 101.f) || !(w.bui >= 0.f) || !(w.ws_kmh >= 0.f) || !std::isfinite(w.bui) ||
            !std::isfinite(w.ws_kmh) || !std::isfinite(w.wd_deg_from))
            return fail(ctx, C2F_EINVAL, "weather row %lld out of range", (long long)i);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    Weather W;
    W.n_scen = n_scen;
    W.n_periods = n_periods;
    W.period_min = period_min;
    c2f_status st;
    if ((st = dev_alloc(ctx, (void**)&W.rows, (size_t)nr * 16)) != C2F_OK) return st;
    if ((st = dev_alloc(ctx, (void**)&W.t64, (size_t)nr * kRowLen * 8)) != C2F_OK) {
        dev_free(ctx, W.rows, (size_t)nr * 16);
        return st;
    }
    if ((st = dev_alloc(ctx, (void**)&W.t32, (size_t)nr * kRowLen * 4)) != C2F_OK) {
        dev_free(ctx, W.rows, (size_t)nr * 16);
        dev_free(ctx, W.t64, (size_t)nr * kRowLen * 8);
        return st;
    }
    hipError_t e = hipMemcpyAsync(W.rows, rows, (size_t)nr * 16, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = launch_weather_table(W.rows, (int)nr, W.t64, W.t32, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        dev_free(ctx, W.rows, (size_t)nr * 16);
        dev_free(ctx, W.t64, (size_t)nr * kRowLen * 8);
        dev_free(ctx, W.t32, (size_t)nr * kRowLen * 4);
        return fail(ctx, C2F_EDEVICE, "weather upload failed: %s", hipGetErrorString(e));
    }
    W.bytes = (size_t)nr * (16 + kRowLen * 12);
    const int32_t id = ctx->next_id++;
    ctx->weathers[id] = W;
    *weather_id = id;
    return C2F_OK;
}

c2f_status c2f_unset_weather(c2f_ctx* ctx, int32_t weather_id) {
    if (!ctx) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
    auto it = ctx->weathers.find(weather_id);
    if (it == ctx->weathers.end()) return fail(ctx, C2F_ESTATE, "unknown weather id %d", weather_id);
    (void)hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
    Weather& W = it->second;
    const size_t nr = (size_t)W.n_scen * W.n_periods;
    dev_free(ctx, W.rows, nr * 16);
    dev_free(ctx, W.t64, nr * kRowLen * 8);
    dev_free(ctx, W.t32, nr * kRowLen * 4);
    ctx->weathers.erase(it);
    return C2F_OK;
}

c2f_status c2f_simulate(c2f_ctx* ctx, const c2f_sim_params* params, const c2f_outputs* out) {
    if (!ctx) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
    ctx->err.clear();
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, C2F_EDEVICE, "hipSetDevice failed");
    return simulate_impl(ctx, 1, params, out, true);
}

c2f_status c2f_simulate_batch(c2f_ctx* ctx, int32_t n_jobs, const c2f_sim_params* params, const c2f_outputs* out) {
    if (!ctx) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
    ctx->err.clear();
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, C2F_EDEVICE, "hipSetDevice failed");
    return simulate_impl(ctx, n_jobs, params, out, true);
}

c2f_status c2f_eval_ros(c2f_ctx* ctx, int32_t landscape_id, int32_t weather_id, int32_t scenario, int32_t period,
                        int32_t rep, uint64_t seed, float sigma, int32_t rounding, int32_t precision, double* hros,
                        double* bros, double* fros, double* lb, double* raz_deg, double* x8, int32_t* q8) {
    if (!ctx) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
    ctx->err.clear();
    auto li = ctx->lands.find(landscape_id);
    if (li == ctx->lands.end()) return fail(ctx, C2F_ESTATE, "unknown landscape id %d", landscape_id);
    auto wi = ctx->weathers.find(weather_id);
    if (wi == ctx->weathers.end()) return fail(ctx, C2F_ESTATE, "unknown weather id %d", weather_id);
    const Landscape& L = li->second;
    const Weather& W = wi->second;
    if (scenario < 0 || scenario >= W.n_scen || period < 0 || period >= W.n_periods || rep < 0)
        return fail(ctx, C2F_EINVAL, "scenario/period/rep out of range");
    if (!(sigma >= 0.f) || !std::isfinite(sigma) || (rounding != 0 && rounding != 1) ||
        (precision != 0 && precision != 1))
        return fail(ctx, C2F_EINVAL, "bad sigma/rounding/precision");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const size_t n = (size_t)L.ncells();
    const size_t bytes = n * 8 * 5 + n * 64 + n * 32 + 7 * 256;   // 7 arrays, 256-byte aligned
    c2f_status st = ensure_staging(ctx, bytes);
    if (st != C2F_OK) return st;
    char* sb = (char*)ctx->staging;
    EvalArgs a;
    memset(&a, 0, sizeof a);
    a.cells = L.cells;
    a.land = L.land;
    a.table = precision == 1 ? (const void*)W.t32 : (const void*)W.t64;
    a.table64 = W.t64;
    a.n_cells = (int32_t)n;
    a.scenario = scenario;
    a.period = period;
    a.n_wp = W.n_periods;
    a.rep = (uint32_t)rep;
    a.rounding = rounding;
    a.sigma = sigma;
    a.seed = seed;
    size_t off = 0;
    auto take = [&](size_t b) {
        char* p = sb + off;
        off += (b + 255) & ~(size_t)255;
        return p;
    };
    a.hros = hros ? (double*)take(n * 8) : nullptr;
    a.bros = bros ? (double*)take(n * 8) : nullptr;
    a.fros = fros ? (double*)take(n * 8) : nullptr;
    a.lb = lb ? (double*)take(n * 8) : nullptr;
    a.raz = raz_deg ? (double*)take(n * 8) : nullptr;
    a.x8 = x8 ? (double*)take(n * 64) : nullptr;
    a.q8 = q8 ? (int32_t*)take(n * 32) : nullptr;
    HIP_TRY(ctx, launch_eval_ros(precision, a, ctx->stream));
    if (hros) HIP_TRY(ctx, hipMemcpyAsync(hros, a.hros, n * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (bros) HIP_TRY(ctx, hipMemcpyAsync(bros, a.bros, n * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (fros) HIP_TRY(ctx, hipMemcpyAsync(fros, a.fros, n * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (lb) HIP_TRY(ctx, hipMemcpyAsync(lb, a.lb, n * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (raz_deg) HIP_TRY(ctx, hipMemcpyAsync(raz_deg, a.raz, n * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (x8) HIP_TRY(ctx, hipMemcpyAsync(x8, a.x8, n * 64, hipMemcpyDeviceToHost, ctx->stream));
    if (q8) HIP_TRY(ctx, hipMemcpyAsync(q8, a.q8, n * 32, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return C2F_OK;
}

c2f_status c2f_fbp_coefficients(int32_t fuel, double out5[5]) {
    static const FuelCoef table[kNumFuels] = {C2F_FUEL_ROWS};
    if (fuel < 1 || fuel > 15 || !out5) return C2F_EINVAL;
    out5[0] = table[fuel].a;
    out5[1] = table[fuel].b;
    out5[2] = table[fuel].c;
    out5[3] = table[fuel].q;
    out5[4] = table[fuel].bui0;
    return C2F_OK;
}

c2f_status c2f_set_tuning(c2f_ctx* ctx, int32_t block_threads, int64_t list_capacity) {
    if (!ctx) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
    if (block_threads != 0 && block_threads != 64 && block_threads != 128 && block_threads != 256 &&
        block_threads != 512 && block_threads != 1024)
        return fail(ctx, C2F_EINVAL, "block_threads must be 0 or one of 64,128,256,512,1024");
    if (list_capacity < 0 || list_capacity > ((int64_t)1 << 30))
        return fail(ctx, C2F_EINVAL, "list_capacity out of range");
    ctx->block_override = block_threads;
    ctx->cap_override = list_capacity;
    return C2F_OK;
}

c2f_status c2f_autotune(c2f_ctx* ctx, const c2f_sim_params* rep) {
    if (!ctx) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
    ctx->err.clear();
    const Landscape* L;
    const Weather* W;
    c2f_status st = check_params(ctx, rep, &L, &W);
    if (st != C2F_OK) return st;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int64_t n = L->ncells();
    uint32_t* counts = nullptr;
    st = dev_alloc(ctx, (void**)&counts, (size_t)n * 4);
    if (st != C2F_OK) return st;
    c2f_outputs o;
    memset(&o, 0, sizeof o);
    o.burn_count = counts;
    o.on_device = 1;
    const int32_t saved_block = ctx->block_override;
    const int64_t saved_cap = ctx->cap_override;
    // first run at the default settings finds the list high-water mark
    ctx->block_override = 0;
    ctx->cap_override = 0;
    st = simulate_impl(ctx, 1, rep, &o, false);
    int64_t cap = ctx->last.list_capacity;
    const int64_t hw = (int64_t)ctx->rc_host->c[kCntMaxList];
    if (st == C2F_OK && hw > 0) cap = std::max<int64_t>(1024, std::min<int64_t>(cap, 4 * hw));
    int32_t best_block = 256;
    double best_ms = 1e30;
    const int blocks[5] = {64, 128, 256, 512, 1024};
    for (int b = 0; b < 5 && st == C2F_OK; ++b) {
        ctx->block_override = blocks[b];
        ctx->cap_override = cap;
        double ms_sum = 0;
        for (int t = 0; t < 2 && st == C2F_OK; ++t) {
            st = simulate_impl(ctx, 1, rep, &o, false);
            ms_sum += ctx->last.kernel_ms;
            if (ctx->last.relaunches) cap = ctx->last.list_capacity;
        }
        if (st == C2F_OK && ms_sum < best_ms) {
            best_ms = ms_sum;
            best_block = blocks[b];
        }
    }
    ctx->block_override = saved_block;
    ctx->cap_override = saved_cap;
    dev_free(ctx, counts, (size_t)n * 4);
    if (st != C2F_OK) return st;
    ctx->tune[TuneKey{n, rep->reps, rep->precision}] = TuneVal{best_block, cap};
    return C2F_OK;
}

c2f_status c2f_get_stats(const c2f_ctx* ctx, c2f_run_stats* out) {
    if (!ctx || !out) return C2F_EINVAL;
    *out = ctx->last;
    return C2F_OK;
}

// ------------------------------------------------------------- serving

c2f_status c2f_submit(c2f_ctx* ctx, const c2f_sim_params* params, const c2f_outputs* out, uint64_t* ticket) {
    if (!ctx || !params || !out || !ticket) return C2F_EINVAL;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
        const Landscape* L;
        const Weather* W;
        c2f_status st = check_params(ctx, params, &L, &W);
        if (st != C2F_OK) return st;
    }
    auto t = std::make_shared<Ticket>();
    t->params = *params;
    t->out = *out;
    {
        std::lock_guard<std::mutex> lk(ctx->smu);
        if ((int32_t)ctx->queue.size() >= ctx->max_queue) return fail(ctx, C2F_EBUSY, "serving queue full");
        t->id = ctx->next_ticket++;
        ctx->tickets[t->id] = t;
        ctx->queue.push_back(t);
        if (!ctx->server.joinable()) ctx->server = std::thread(server_loop, ctx);
    }
    ctx->scv.notify_all();
    *ticket = t->id;
    return C2F_OK;
}

c2f_status c2f_poll(c2f_ctx* ctx, uint64_t ticket, int32_t* done) {
    if (!ctx || !done) return C2F_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->smu);
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return C2F_ESTATE;
    *done = it->second->done ? 1 : 0;
    return C2F_OK;
}

c2f_status c2f_wait(c2f_ctx* ctx, uint64_t ticket) {
    if (!ctx) return C2F_EINVAL;
    std::unique_lock<std::mutex> lk(ctx->smu);
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return C2F_ESTATE;
    std::shared_ptr<Ticket> t = it->second;
    ctx->scv.wait(lk, [&] { return t->done; });
    const c2f_status st = t->status;
    if (st != C2F_OK) ctx->err = t->err;
    ctx->tickets.erase(ticket);
    return st;
}

}  // extern "C"

namespace {

// Serving loop: take every waiting request whose memory fits, run them as
// one fused launch, complete their tickets, repeat.  Requests that arrive
// while a batch is on the device join the next batch.
void server_loop(c2f_ctx* ctx) {
    (void)hipSetDevice(ctx->device);
    for (;;) {
        std::vector<std::shared_ptr<Ticket>> batch;
        {
            std::unique_lock<std::mutex> lk(ctx->smu);
            ctx->scv.wait(lk, [&] { return ctx->stopping || !ctx->queue.empty(); });
            if (ctx->stopping && ctx->queue.empty()) return;
            int64_t items = 0;
            while (!ctx->queue.empty()) {
                auto& t = ctx->queue.front();
                if (!batch.empty() && items + t->params.reps > ctx->max_batch_items) break;
                items += t->params.reps;
                batch.push_back(t);
                ctx->queue.pop_front();
            }
        }
        std::vector<c2f_sim_params> P;
        std::vector<c2f_outputs> O;
        for (auto& t : batch) {
            P.push_back(t->params);
            O.push_back(t->out);
        }
        c2f_status st;
        std::string err;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
    clear_sticky_error();
            st = simulate_impl(ctx, (int32_t)P.size(), P.data(), O.data(), false);
            err = ctx->err;
            if (st != C2F_OK && P.size() > 1) {
                // run one by one so a bad request only fails itself
                for (size_t k = 0; k < P.size(); ++k) {
                    c2f_status s1 = simulate_impl(ctx, 1, &P[k], &O[k], false);
                    std::lock_guard<std::mutex> lk2(ctx->smu);
                    batch[k]->status = s1;
                    batch[k]->err = ctx->err;
                }
            }
        }
        {
            std::lock_guard<std::mutex> lk(ctx->smu);
            for (auto& t : batch) {
                if (!(st != C2F_OK && P.size() > 1)) {
                    t->status = st;
                    t->err = err;
                }
                t->done = true;
            }
        }
        ctx->scv.notify_all();
    }
}

}  // namespace
