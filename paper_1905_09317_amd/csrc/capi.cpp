// libc2f host runtime: device memory, executors (a stream with its work
// slots, lists, counters and staging), relaunch on work-list overflow,
// batching of requests into one launch, hipGraph replay, autotuning, and the
// serving lanes that run admitted batches concurrently.  Implements
// include/c2f.h.

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

// Message of the most recent failure on the calling thread; copied into the
// context's error text when an entry point returns.
thread_local std::string t_err;

struct Landscape {
    int32_t rows = 0, cols = 0, cell_m = 0;
    float pc = 50.f, curing = 80.f;
    float fmc = 97.f, pdf = 50.f;   // foliar moisture content, percent dead fir
    uint8_t* fuel = nullptr;
    CellRec* cells = nullptr;
    int32_t* burnable = nullptr;
    LandDev* land = nullptr;
    uint64_t* ign_cdf = nullptr;   // ignition map: running weight sums (device)
    uint64_t ign_total = 0;
    int32_t inflight = 0;   // submitted requests not yet completed
    int64_t ncells() const { return (int64_t)rows * cols; }
};

struct Weather {
    int32_t n_scen = 0, n_periods = 0, period_min = 0;
    float* rows = nullptr;
    double* t64 = nullptr;
    float* t32 = nullptr;
    int32_t inflight = 0;
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

// An executor: one HIP stream and the device buffers its launches use.
// Buffers only grow; a serving lane rounds sizes up to powers of two so that
// batches of varying shape rarely reallocate.
struct Exec {
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    bool round_up = false;

    uint32_t* planes = nullptr;   // n_slots x plane_cells arrival labels
    int64_t plane_cells = 0;
    int32_t n_slots = 0;
    // Serving lanes hold one plane pool and lay the slots out inside it per
    // launch (plane_cells = the launch's rounded grid size); the first
    // tag_ready slots hold planes and tags valid for that layout.
    size_t plane_pool = 0;
    int32_t tag_ready = 0;
    size_t list_pool = 0;         // serving lanes: bytes held for the lists, laid out per launch
    uint8_t* lists = nullptr;     // list_slots x list_cap x kSlotListBytesPerEntry
    int64_t list_cap = 0;
    int32_t list_slots = 0;
    uint32_t* tags = nullptr;     // tag_slots generation tags
    int32_t tag_slots = 0;

    RunCounters* rc = nullptr;
    RunCounters* rc_host = nullptr;   // pinned
    Job* d_jobs = nullptr;
    int32_t d_jobs_cap = 0;
    Job* h_jobs = nullptr;            // pinned
    int32_t h_jobs_cap = 0;

    void* staging = nullptr;          // device copy of host-bound outputs
    size_t staging_bytes = 0;
    void* host_stage = nullptr;       // pinned host copy of the same, read by memcpy
    size_t host_stage_bytes = 0;
    int2* item_slot = nullptr;        // {slot, tag} per item of a launch
    int32_t item_slot_cap = 0;
    unsigned long long* order_keys = nullptr;   // replication order: a key
    int32_t* order = nullptr;                   // and a position per item
    int32_t order_cap = 0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    c2f_run_stats last{};

    // hipGraph of the last launch sequence (synchronous calls only)
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<uint64_t> graph_key;
    bool graph_unavailable = false;   // capture refused once: launch eagerly
};

struct Ticket {
    uint64_t id = 0;
    c2f_sim_params params{};
    std::vector<int32_t> ign_list;   // the request's ignition-point list, copied
    c2f_outputs out{};
    Landscape* L = nullptr;
    Weather* W = nullptr;
    bool done = false;
    c2f_status status = C2F_OK;
    std::string err;
    c2f_ticket_info info{};
};

struct Lane {
    Exec ex;
    std::thread th;
    bool busy = false;
    int32_t index = 0;
};

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct c2f_ctx {
    int device = 0;
    uint64_t budget = 0;        // caller's cap on device bytes (0 = none)
    uint64_t admit_limit = 0;   // bytes serving admission plans against
    size_t lane_plane_budget = 0;   // plane pool of one serving lane
    size_t lane_list_budget = 0;    // list pool of one serving lane
    int n_cu = 0;
    std::string arch;           // device architecture, e.g. "gfx950" (feature suffixes dropped)
    std::chrono::steady_clock::time_point t0;
    void* scratch = nullptr;    // device address of the no-allocation scratch on `device`
    void* acct = nullptr;       // work counts: 3 counters and a job record (allocated on first use)

    std::mutex errmu;
    std::string err;

    std::mutex mu;   // serialises the synchronous entry points; guards `main` and `metric_buf`
    Exec main;
    void* metric_buf = nullptr;   // scar comparison counts and results, kept between calls
    size_t metric_bytes = 0;
    size_t metric_periods = 0;    // periods metric_buf is laid out for

    // Landscapes and weather.  Inserting or erasing needs `mu` and `objmu`;
    // lookups hold either; the in-flight counts need `objmu`.
    std::mutex objmu;
    std::map<int32_t, Landscape> lands;
    std::map<int32_t, Weather> weathers;
    int32_t next_id = 1;

    std::mutex memmu;   // device-memory ledger
    size_t bytes_in_use = 0;

    std::mutex tunemu;
    int32_t rep_order = 1;    // 1: longest predicted replications first when groups run several
    int32_t block_override = 0;
    int64_t cap_override = 0;
    std::map<TuneKey, TuneVal> tune;

    // serving
    std::mutex smu;
    std::condition_variable scv;
    std::deque<std::shared_ptr<Ticket>> queue;
    std::map<uint64_t, std::shared_ptr<Ticket>> tickets;
    uint64_t next_ticket = 1;
    std::vector<std::unique_ptr<Lane>> lanes;
    int32_t n_lanes = 4;
    int32_t max_queue = 4096;
    int32_t max_batch_reps = 2048;
    int32_t max_batch_grid = 0;
    int32_t busy_lanes = 0;
    size_t promised = 0;   // growth admitted to running lanes, not yet released
    bool stopping = false;
};

namespace {

// Drop any error left by an earlier runtime call whose status was ignored,
// so that launch checks (hipGetLastError) report only their own launch.
inline void clear_sticky_error() { (void)hipGetLastError(); }

c2f_status fail(c2f_ctx*, c2f_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return st;
}

// Scope of one entry point: starts with a clean error state and publishes
// the thread's error text to the context on return.
struct ApiScope {
    c2f_ctx* ctx;
    explicit ApiScope(c2f_ctx* c) : ctx(c) {
        t_err.clear();
        clear_sticky_error();
    }
    ~ApiScope() {
        std::lock_guard<std::mutex> lk(ctx->errmu);
        ctx->err = t_err;
    }
};

#define HIP_TRY(ctx, expr)                                                                         \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((ctx), C2F_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

c2f_status dev_alloc(c2f_ctx* ctx, void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    {
        std::lock_guard<std::mutex> lk(ctx->memmu);
        if (ctx->budget && ctx->bytes_in_use + bytes > ctx->budget)
            return fail(ctx, C2F_ENOMEM, "HBM budget exceeded: %zu in use + %zu requested > %llu",
                        ctx->bytes_in_use, bytes, (unsigned long long)ctx->budget);
        ctx->bytes_in_use += bytes;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        std::lock_guard<std::mutex> lk(ctx->memmu);
        ctx->bytes_in_use -= std::min(ctx->bytes_in_use, bytes);
        return fail(ctx, C2F_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    return C2F_OK;
}

void dev_free(c2f_ctx* ctx, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    if (bytes == 0) bytes = 16;
    std::lock_guard<std::mutex> lk(ctx->memmu);
    ctx->bytes_in_use -= std::min(ctx->bytes_in_use, bytes);
}

size_t bytes_in_use(c2f_ctx* ctx) {
    std::lock_guard<std::mutex> lk(ctx->memmu);
    return ctx->bytes_in_use;
}

int32_t axis_diag(int32_t cs) {
    // least integer D with D*D >= 2 cs^2
    const int64_t two = 2ll * cs * cs;
    int64_t d = (int64_t)std::sqrt((double)two);
    while (d * d < two) ++d;
    while ((d - 1) * (d - 1) >= two) --d;
    return (int32_t)d;
}

int64_t pow2_at_least(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// ---------------------------------------------------------------- executors

void drop_graph(Exec& ex) {
    if (ex.graph_exec) (void)hipGraphExecDestroy(ex.graph_exec);
    if (ex.graph) (void)hipGraphDestroy(ex.graph);
    clear_sticky_error();
    ex.graph_exec = nullptr;
    ex.graph = nullptr;
    ex.graph_key.clear();
}

// The main executor's own stream is a blocking stream, ordered with the
// legacy null stream both ways (callers such as torch's default stream see
// library writes in order); serving lanes use non-blocking streams and
// complete their requests before reporting them done.
c2f_status exec_init(c2f_ctx* ctx, Exec& ex, bool lane) {
    ex.round_up = lane;
    HIP_TRY(ctx, hipStreamCreateWithFlags(&ex.own_stream, lane ? hipStreamNonBlocking : hipStreamDefault));
    ex.stream = ex.own_stream;
    HIP_TRY(ctx, hipEventCreate(&ex.ev0));
    HIP_TRY(ctx, hipEventCreate(&ex.ev1));
    c2f_status st = dev_alloc(ctx, (void**)&ex.rc, sizeof(RunCounters));
    if (st != C2F_OK) return st;
    HIP_TRY(ctx, hipHostMalloc((void**)&ex.rc_host, sizeof(RunCounters), hipHostMallocDefault));
    return C2F_OK;
}

// Free the growable buffers (planes, lists, tags, staging, job table).
void exec_trim(c2f_ctx* ctx, Exec& ex) {
    if (ex.stream) (void)hipStreamSynchronize(ex.stream);
    drop_graph(ex);
    dev_free(ctx, ex.planes, ex.round_up ? ex.plane_pool : (size_t)ex.n_slots * ex.plane_cells * 4);
    dev_free(ctx, ex.lists,
             ex.round_up ? ex.list_pool : (size_t)ex.list_slots * ex.list_cap * kSlotListBytesPerEntry);
    dev_free(ctx, ex.tags, (size_t)ex.tag_slots * 4);
    dev_free(ctx, ex.staging, ex.staging_bytes);
    dev_free(ctx, ex.d_jobs, (size_t)ex.d_jobs_cap * sizeof(Job));
    dev_free(ctx, ex.item_slot, (size_t)ex.item_slot_cap * sizeof(int2));
    ex.item_slot = nullptr;
    ex.item_slot_cap = 0;
    dev_free(ctx, ex.order_keys, (size_t)ex.order_cap * kOrderBytesPerItem);
    ex.order_keys = nullptr;
    ex.order = nullptr;
    ex.order_cap = 0;
    ex.planes = nullptr;
    ex.n_slots = 0;
    ex.plane_cells = 0;
    ex.plane_pool = 0;
    ex.tag_ready = 0;
    ex.list_pool = 0;
    if (ex.host_stage) (void)hipHostFree(ex.host_stage);
    ex.host_stage = nullptr;
    ex.host_stage_bytes = 0;
    ex.lists = nullptr;
    ex.list_slots = 0;
    ex.list_cap = 0;
    ex.tags = nullptr;
    ex.tag_slots = 0;
    ex.staging = nullptr;
    ex.staging_bytes = 0;
    ex.d_jobs = nullptr;
    ex.d_jobs_cap = 0;
}

void exec_release(c2f_ctx* ctx, Exec& ex) {
    exec_trim(ctx, ex);
    dev_free(ctx, ex.rc, sizeof(RunCounters));
    ex.rc = nullptr;
    if (ex.h_jobs) (void)hipHostFree(ex.h_jobs);
    if (ex.rc_host) (void)hipHostFree(ex.rc_host);
    if (ex.ev0) (void)hipEventDestroy(ex.ev0);
    if (ex.ev1) (void)hipEventDestroy(ex.ev1);
    if (ex.own_stream) (void)hipStreamDestroy(ex.own_stream);
    ex.h_jobs = nullptr;
    ex.h_jobs_cap = 0;
    ex.rc_host = nullptr;
    ex.ev0 = ex.ev1 = nullptr;
    ex.own_stream = ex.stream = nullptr;
}

// Sizes the slot buffers of `ex` must have to run n slots of `cells` labels
// with lists of at least `cap` entries.
struct SlotSizes {
    int32_t n_slots;
    int64_t plane_cells;
    int32_t list_slots;
    int64_t list_cap;
    bool grow_planes, grow_lists;
};

SlotSizes slot_sizes(const Exec& ex, int32_t n, int64_t cells, int64_t cap) {
    if (ex.round_up) {
        n = (int32_t)pow2_at_least(n);
        cells = pow2_at_least(cells);
        cap = pow2_at_least(cap);
    }
    SlotSizes s;
    s.grow_planes = n > ex.n_slots || cells > ex.plane_cells;
    s.n_slots = std::max(n, ex.n_slots);
    s.plane_cells = std::max(cells, ex.plane_cells);
    s.grow_lists = n > ex.list_slots || cap > ex.list_cap;
    s.list_slots = std::max(n, ex.list_slots);
    s.list_cap = std::max(cap, ex.list_cap);
    return s;
}

// Plane pool a serving lane allocates to run n slots of `cells`: the lane's
// share of the serving memory, or more when a single launch needs it.
size_t lane_pool_bytes(size_t budget, int32_t n, int64_t cells) {
    return std::max(budget, (size_t)n * (size_t)pow2_at_least(cells) * 4);
}

// Slots a serving lane runs for grids of `cells`: as many as its plane pool
// holds (at least one).
int32_t lane_slot_cap(size_t budget, int64_t cells) {
    const size_t per = (size_t)pow2_at_least(cells) * 4;
    return (int32_t)std::max<size_t>(1, std::min<size_t>(budget / per, (size_t)1 << 20));
}

// List capacity a serving lane gives each of n slots: the launch's plan,
// at most what its list pool holds (an overflow still relaunches larger).
int64_t lane_list_cap(size_t list_budget, int32_t n, int64_t cap) {
    int64_t fit = (int64_t)(list_budget / ((size_t)std::max(n, 1) * kSlotListBytesPerEntry));
    fit = std::max<int64_t>(fit, 4096);
    int64_t c = pow2_at_least(cap);
    while (c > fit && c > 4096) c >>= 1;
    return c;
}

// Device bytes `ex` would add to run n slots of `cells` with lists of
// `cap` entries, `stage` bytes of output staging and n_jobs requests
// (`budget`, `list_budget`: a serving lane's plane and list pools).
size_t exec_growth(const Exec& ex, int32_t n, int64_t cells, int64_t cap, size_t stage, int32_t n_jobs,
                   size_t budget, size_t list_budget) {
    const SlotSizes s = slot_sizes(ex, n, cells, cap);
    size_t g = 0;
    if (n_jobs > ex.d_jobs_cap)
        g += ((size_t)pow2_at_least(std::max(n_jobs, 64)) - (size_t)ex.d_jobs_cap) * sizeof(Job);
    if (ex.round_up) {
        const size_t need = (size_t)n * (size_t)pow2_at_least(cells) * 4;
        if (need > ex.plane_pool) g += lane_pool_bytes(budget, n, cells) - ex.plane_pool;
        if (n > ex.tag_slots) g += ((size_t)pow2_at_least(n) - (size_t)ex.tag_slots) * 4;
        const size_t lneed = (size_t)n * (size_t)pow2_at_least(cap) * kSlotListBytesPerEntry;
        if (lneed > ex.list_pool) g += std::max(lneed, list_budget) - ex.list_pool;
    } else if (s.grow_planes) {
        g += (size_t)s.n_slots * s.plane_cells * 4 - (size_t)ex.n_slots * ex.plane_cells * 4;
        g += (size_t)s.n_slots * 4;
    }
    if (!ex.round_up && s.grow_lists)
        g += (size_t)s.list_slots * s.list_cap * kSlotListBytesPerEntry -
             (size_t)ex.list_slots * ex.list_cap * kSlotListBytesPerEntry;
    const size_t stage_alloc = ex.round_up && stage ? (size_t)pow2_at_least((int64_t)stage) : stage;
    if (stage_alloc > ex.staging_bytes) g += stage_alloc - ex.staging_bytes;
    if (n > ex.item_slot_cap) g += ((size_t)pow2_at_least(std::max(n, 64)) - (size_t)ex.item_slot_cap) * sizeof(int2);
    return g;
}

c2f_status ensure_slots(c2f_ctx* ctx, Exec& ex, int32_t n, int64_t cells, int64_t cap) {
    const SlotSizes s = slot_sizes(ex, n, cells, cap);
    if (ex.round_up) {
        // Serving lane: one plane pool, allocated once (or when a single
        // launch needs more); slots are laid out at the launch's rounded
        // grid size, and a slot whose plane holds another layout's labels
        // starts from an exhausted tag, so that its work group refills the
        // plane before its first replication.
        const int64_t stride = pow2_at_least(cells);
        const size_t need = (size_t)n * (size_t)stride * 4;
        if (need > ex.plane_pool) {
            drop_graph(ex);
            dev_free(ctx, ex.planes, ex.plane_pool);
            ex.planes = nullptr;
            ex.plane_pool = 0;
            ex.tag_ready = 0;
            const size_t pool = lane_pool_bytes(ctx->lane_plane_budget, n, cells);
            c2f_status st = dev_alloc(ctx, (void**)&ex.planes, pool);
            if (st != C2F_OK) return st;
            ex.plane_pool = pool;
        }
        if (n > ex.tag_slots) {
            drop_graph(ex);
            dev_free(ctx, ex.tags, (size_t)ex.tag_slots * 4);
            ex.tags = nullptr;
            ex.tag_slots = 0;
            ex.tag_ready = 0;
            const int32_t nt = (int32_t)pow2_at_least(n);
            c2f_status st = dev_alloc(ctx, (void**)&ex.tags, (size_t)nt * 4);
            if (st != C2F_OK) return st;
            ex.tag_slots = nt;
        }
        if (stride != ex.plane_cells) {
            ex.plane_cells = stride;
            ex.tag_ready = 0;
        }
        if (n > ex.tag_ready) {
            HIP_TRY(ctx, launch_fill_u32(ex.tags + ex.tag_ready, (size_t)(n - ex.tag_ready), 0u, ex.stream));
            ex.tag_ready = n;
        }
        ex.n_slots = std::max(ex.n_slots, n);
        // lists: one pool as well, laid out per launch (they need no
        // initial contents)
        const int64_t lcap = pow2_at_least(cap);
        const size_t lneed = (size_t)n * (size_t)lcap * kSlotListBytesPerEntry;
        if (lneed > ex.list_pool) {
            drop_graph(ex);
            dev_free(ctx, ex.lists, ex.list_pool);
            ex.lists = nullptr;
            ex.list_pool = 0;
            const size_t pool = std::max(lneed, ctx->lane_list_budget);
            c2f_status st = dev_alloc(ctx, (void**)&ex.lists, pool);
            if (st != C2F_OK) return st;
            ex.list_pool = pool;
        }
        ex.list_cap = lcap;
        ex.list_slots = n;
        return C2F_OK;
    } else if (s.grow_planes) {
        drop_graph(ex);
        dev_free(ctx, ex.planes, (size_t)ex.n_slots * ex.plane_cells * 4);
        ex.planes = nullptr;
        ex.n_slots = 0;
        ex.plane_cells = 0;
        c2f_status st = dev_alloc(ctx, (void**)&ex.planes, (size_t)s.n_slots * s.plane_cells * 4);
        if (st != C2F_OK) return st;
        ex.n_slots = s.n_slots;
        ex.plane_cells = s.plane_cells;
        HIP_TRY(ctx, launch_fill_u32(ex.planes, (size_t)s.n_slots * s.plane_cells, kPlaneFill, ex.stream));
        // every slot restarts from a freshly filled plane
        dev_free(ctx, ex.tags, (size_t)ex.tag_slots * 4);
        ex.tags = nullptr;
        ex.tag_slots = 0;
        st = dev_alloc(ctx, (void**)&ex.tags, (size_t)s.n_slots * 4);
        if (st != C2F_OK) return st;
        ex.tag_slots = s.n_slots;
        HIP_TRY(ctx, launch_fill_u32(ex.tags, (size_t)s.n_slots, kTagFresh, ex.stream));
    }
    if (s.grow_lists) {
        drop_graph(ex);
        dev_free(ctx, ex.lists, (size_t)ex.list_slots * ex.list_cap * kSlotListBytesPerEntry);
        ex.lists = nullptr;
        ex.list_slots = 0;
        ex.list_cap = 0;
        c2f_status st = dev_alloc(ctx, (void**)&ex.lists, (size_t)s.list_slots * s.list_cap * kSlotListBytesPerEntry);
        if (st != C2F_OK) return st;
        ex.list_slots = s.list_slots;
        ex.list_cap = s.list_cap;
    }
    return C2F_OK;
}

c2f_status ensure_jobs(c2f_ctx* ctx, Exec& ex, int32_t n) {
    if (n > ex.d_jobs_cap) {
        drop_graph(ex);
        dev_free(ctx, ex.d_jobs, (size_t)ex.d_jobs_cap * sizeof(Job));
        ex.d_jobs = nullptr;
        ex.d_jobs_cap = 0;
        const int32_t cap = (int32_t)pow2_at_least(std::max(n, 64));
        c2f_status st = dev_alloc(ctx, (void**)&ex.d_jobs, (size_t)cap * sizeof(Job));
        if (st != C2F_OK) return st;
        ex.d_jobs_cap = cap;
    }
    if (n > ex.h_jobs_cap) {
        if (ex.h_jobs) (void)hipHostFree(ex.h_jobs);
        ex.h_jobs = nullptr;
        ex.h_jobs_cap = 0;
        const int32_t cap = (int32_t)pow2_at_least(std::max(n, 64));
        HIP_TRY(ctx, hipHostMalloc((void**)&ex.h_jobs, (size_t)cap * sizeof(Job), hipHostMallocDefault));
        ex.h_jobs_cap = cap;
    }
    return C2F_OK;
}

c2f_status ensure_item_slots(c2f_ctx* ctx, Exec& ex, int32_t n) {
    if (n > ex.item_slot_cap) {
        drop_graph(ex);
        dev_free(ctx, ex.item_slot, (size_t)ex.item_slot_cap * sizeof(int2));
        ex.item_slot = nullptr;
        ex.item_slot_cap = 0;
        const int32_t cap = (int32_t)pow2_at_least(std::max(n, 64));
        c2f_status st = dev_alloc(ctx, (void**)&ex.item_slot, (size_t)cap * sizeof(int2));
        if (st != C2F_OK) return st;
        ex.item_slot_cap = cap;
    }
    return C2F_OK;
}

// Key and position per item for the replication order (one allocation).
c2f_status ensure_order(c2f_ctx* ctx, Exec& ex, int32_t n) {
    if (n > ex.order_cap) {
        drop_graph(ex);
        dev_free(ctx, ex.order_keys, (size_t)ex.order_cap * kOrderBytesPerItem);
        ex.order_keys = nullptr;
        ex.order = nullptr;
        ex.order_cap = 0;
        const int32_t cap = (int32_t)pow2_at_least(std::max(n, 64));
        c2f_status st = dev_alloc(ctx, (void**)&ex.order_keys, (size_t)cap * kOrderBytesPerItem);
        if (st != C2F_OK) return st;
        ex.order = (int32_t*)(ex.order_keys + cap);
        ex.order_cap = cap;
    }
    return C2F_OK;
}

c2f_status ensure_staging(c2f_ctx* ctx, Exec& ex, size_t bytes) {
    if (bytes > ex.staging_bytes) {
        drop_graph(ex);
        dev_free(ctx, ex.staging, ex.staging_bytes);
        ex.staging = nullptr;
        ex.staging_bytes = 0;
        const size_t alloc = ex.round_up ? (size_t)pow2_at_least((int64_t)bytes) : bytes;
        c2f_status st = dev_alloc(ctx, &ex.staging, alloc);
        if (st != C2F_OK) return st;
        ex.staging_bytes = alloc;
    }
    return C2F_OK;
}

// Pinned host memory the device staging is copied into in one transfer;
// the host then copies each output to the caller's (possibly pageable)
// buffer.  A device-to-pageable copy goes through the runtime's own bounce
// buffer in pieces and serialises concurrent lanes.
c2f_status ensure_host_stage(c2f_ctx* ctx, Exec& ex, size_t bytes) {
    if (bytes > ex.host_stage_bytes) {
        if (ex.host_stage) (void)hipHostFree(ex.host_stage);
        ex.host_stage = nullptr;
        ex.host_stage_bytes = 0;
        const size_t alloc = ex.round_up ? (size_t)pow2_at_least((int64_t)bytes) : bytes;
        if (hipHostMalloc(&ex.host_stage, alloc, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            ex.host_stage = nullptr;
            return fail(ctx, C2F_ENOMEM, "pinned host staging of %zu bytes failed", alloc);
        }
        ex.host_stage_bytes = alloc;
    }
    return C2F_OK;
}

// ---------------------------------------------------------------- requests

c2f_status check_params(c2f_ctx* ctx, const c2f_sim_params* p, Landscape** L, Weather** W) {
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
    if (p->ignition_mode < 0 || p->ignition_mode > 4) return fail(ctx, C2F_EINVAL, "ignition_mode must be 0..4");
    if (p->ignition_mode == 4) {
        if (p->n_ignitions < 1 || p->n_ignitions > kMaxIgnitions || !p->ignition_list)
            return fail(ctx, C2F_EINVAL, "ignition_mode 4 needs 1..%d (cell, period) pairs in ignition_list",
                        kMaxIgnitions);
        for (int32_t k = 0; k < p->n_ignitions; ++k) {
            const int32_t c = p->ignition_list[2 * k], q = p->ignition_list[2 * k + 1];
            if (c < 0 || c >= l.ncells())
                return fail(ctx, C2F_EINVAL, "ignition_list entry %d: cell %d outside the grid", k, c);
            if (q < 0 || q >= p->n_periods)
                return fail(ctx, C2F_EINVAL, "ignition_list entry %d: period %d not in 0..%d", k, q,
                            p->n_periods - 1);
        }
    } else if (p->n_ignitions != 0) {
        return fail(ctx, C2F_EINVAL, "n_ignitions > 0 needs ignition_mode 4");
    }
    if (p->ignition_mode == 3 && !l.ign_cdf)
        return fail(ctx, C2F_EINVAL, "ignition_mode 3 needs an ignition map (c2f_set_ignition_map)");
    if (p->ignition_period < 0 || p->ignition_period >= p->n_periods)
        return fail(ctx, C2F_EINVAL, "ignition_period %d not in 0..%d", p->ignition_period, p->n_periods - 1);
    if (p->burn_hours < 0 || p->burn_hours > 24) return fail(ctx, C2F_EINVAL, "burn_hours must be 0..24");
    if (!(p->burnout_ros >= 0.f) || !std::isfinite(p->burnout_ros))
        return fail(ctx, C2F_EINVAL, "burnout_ros must be finite and >= 0");
    if (!(p->hfi_min >= 0.f) || !std::isfinite(p->hfi_min))
        return fail(ctx, C2F_EINVAL, "hfi_min must be finite and >= 0");
    if (p->burn_hours > 0 && p->burn_hours < 24 && (w.period_min > 60 || 60 % w.period_min != 0))
        return fail(ctx, C2F_EINVAL, "burn_hours needs a period length dividing 60 minutes (got %d)",
                    w.period_min);
    if (p->ignition_mode == 0 && (p->ignition_cell < 0 || p->ignition_cell >= l.ncells()))
        return fail(ctx, C2F_EINVAL, "ignition_cell %d outside the grid", p->ignition_cell);
    if (p->scenario_mode < 0 || p->scenario_mode > 1) return fail(ctx, C2F_EINVAL, "scenario_mode must be 0 or 1");
    if (p->scenario_mode == 0 && (p->scenario < 0 || p->scenario >= w.n_scen))
        return fail(ctx, C2F_EINVAL, "scenario %d not in 0..%d", p->scenario, w.n_scen - 1);
    *L = &li->second;
    *W = &wi->second;
    return C2F_OK;
}

int64_t default_list_cap(int64_t cells, int32_t reps) {
    // Generous for single large fires, modest when many slots share HBM;
    // an overflow is detected and the run repeated with a larger capacity.
    int64_t cap = reps <= 64 ? (int64_t)1 << 20 : (int64_t)1 << 16;
    cap = std::min<int64_t>(cap, std::max<int64_t>(1024, 2 * cells));
    return cap;
}

struct LaunchPlan {
    int32_t block = 256;
    int32_t grid = 1;
    int64_t cap = 1024;
};

LaunchPlan plan_launch(c2f_ctx* ctx, int64_t cells, int32_t total_items, int32_t precision, int32_t grid_cap) {
    LaunchPlan lp;
    {
        std::lock_guard<std::mutex> lk(ctx->tunemu);
        auto it = ctx->tune.find(TuneKey{cells, total_items, precision});
        if (it != ctx->tune.end()) {
            lp.block = it->second.block;
            lp.cap = it->second.list_cap;
        } else {
            // At most one replication per compute unit on a large grid:
            // wide groups, since nothing else would use the unit.  FP64
            // keeps 512 threads (2 waves per SIMD, 256 VGPRs); at 1024 it
            // would be held to 128 VGPRs and spill (8192^2 x 64 reps: 10.1
            // ms at 512, 12.8 at 256, 18.8 at 1024).  FP32 single fires take
            // 768 threads: 3 waves per SIMD fit the FP32 kernel's 168
            // VGPRs with a 20-byte spill (2048^2 single fire: 3.97 ms at
            // 768, 4.02 at 1024, 4.25 at 512).
            if (cells >= (1 << 20) && total_items <= ctx->n_cu)
                lp.block = (precision == 1 && total_items <= 16) ? 768 : 512;
            else
                lp.block = 256;
            lp.cap = default_list_cap(cells, total_items);
        }
        if (ctx->block_override) lp.block = ctx->block_override;
        if (ctx->cap_override) lp.cap = ctx->cap_override;
    }
    int per_cu = propagate_blocks_per_cu(precision, lp.block);
    if (per_cu < 1) per_cu = 1;
    lp.grid = std::max(1, std::min(total_items, per_cu * ctx->n_cu));
    if (grid_cap > 0) lp.grid = std::min(lp.grid, grid_cap);
    return lp;
}

// The kernel's record of one request: landscape and weather on the device,
// options, and where its outputs go.  Items item_base .. item_base + reps - 1
// of the launch are its replications.
Job make_job(const c2f_sim_params& p, const Landscape& L, const Weather& W, const OutPlan& o,
             int32_t precision, int32_t item) {
    Job j;
    memset(&j, 0, sizeof j);
    j.cells = L.cells;
    j.burnable = L.burnable;
    j.land = L.land;
    j.table = precision == 1 ? (const void*)W.t32 : (const void*)W.t64;
    j.table64 = W.t64;
    j.table32 = W.t32;
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
    j.ign_period = p.ignition_period;
    j.ign_cdf = p.ignition_mode == 3 ? L.ign_cdf : nullptr;
    j.n_seeds = 0;
    if (p.ignition_mode == 4) {
        // the list by period; entries of one period keep their order
        int32_t ord[kMaxIgnitions];
        for (int32_t k = 0; k < p.n_ignitions; ++k) ord[k] = k;
        std::stable_sort(ord, ord + p.n_ignitions, [&](int32_t a, int32_t b) {
            return p.ignition_list[2 * a + 1] < p.ignition_list[2 * b + 1];
        });
        for (int32_t k = 0; k < p.n_ignitions; ++k)
            j.seeds[k] = make_int2(p.ignition_list[2 * ord[k]], p.ignition_list[2 * ord[k] + 1]);
        j.n_seeds = p.n_ignitions;
        j.ign_period = j.seeds[0].y;
    }
    j.ign_total = p.ignition_mode == 3 ? L.ign_total : 0;
    j.burn_hours = (p.burn_hours >= 24) ? 0 : p.burn_hours;
    j.burnout = p.burnout_ros;
    j.hfi_min = p.hfi_min;
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
    return j;
}

// One fused launch over all requests of one precision.  Relaunches with a
// larger list capacity if any work list overflowed.
c2f_status run_group(c2f_ctx* ctx, Exec& ex, const std::vector<int>& idx, const std::vector<c2f_sim_params>& P,
                     const std::vector<const Landscape*>& Ls, const std::vector<const Weather*>& Ws,
                     std::vector<OutPlan>& plans, int32_t precision, bool use_graph, int32_t grid_cap) {
    if (idx.empty()) return C2F_OK;
    int64_t max_cells = 0;
    int32_t total = 0;
    for (int k : idx) {
        max_cells = std::max(max_cells, Ls[k]->ncells());
        total += P[k].reps;
    }
    LaunchPlan lp = plan_launch(ctx, max_cells, total, precision, grid_cap);
    if (ex.round_up) {
        lp.grid = std::min(lp.grid, lane_slot_cap(ctx->lane_plane_budget, max_cells));
        lp.cap = lane_list_cap(std::max(ctx->lane_list_budget, ex.list_pool), lp.grid, lp.cap);
    }
    c2f_status st = ensure_jobs(ctx, ex, (int32_t)idx.size());
    if (st != C2F_OK) return st;
    bool dense = false;
    for (int k : idx) dense |= plans[k].scar || plans[k].arr_minute || plans[k].arr_period;
    int32_t rep_order;
    {
        std::lock_guard<std::mutex> lk(ctx->tunemu);
        rep_order = ctx->rep_order;
    }
    int32_t max_periods = 0;
    for (int k : idx) max_periods = std::max(max_periods, P[k].n_periods);
    for (;;) {
        st = ensure_slots(ctx, ex, lp.grid, max_cells, lp.cap);
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
            ex.h_jobs[q] = make_job(p, L, W, o, precision, item);
            item += p.reps;
        }
        HIP_TRY(ctx, hipMemcpyAsync(ex.d_jobs, ex.h_jobs, idx.size() * sizeof(Job), hipMemcpyHostToDevice,
                                    ex.stream));

        // dense outputs by a grid-wide kernel when no slot runs two items
        const bool defer = dense && total <= lp.grid && total <= 65535;
        if (defer) {
            st = ensure_item_slots(ctx, ex, total);
            if (st != C2F_OK) return st;
        }
        // groups that run several replications take the longest predicted first
        const bool ordered = rep_order == 1 && total > lp.grid && max_periods <= 65535;
        if (ordered) {
            st = ensure_order(ctx, ex, total);
            if (st != C2F_OK) return st;
        }
        const int64_t limit = std::min(lp.cap, ex.list_cap);
        Slots sl{ex.planes,  ex.plane_cells, ex.lists, ex.list_cap, limit, ex.tags, defer ? ex.item_slot : nullptr,
                 ordered ? ex.order : nullptr};
        // key of the launch sequence for graph reuse
        std::vector<uint64_t> key = {(uint64_t)(uintptr_t)ex.d_jobs, idx.size(), (uint64_t)total,
                                     (uint64_t)lp.block, (uint64_t)lp.grid, (uint64_t)precision,
                                     (uint64_t)(uintptr_t)ex.planes, (uint64_t)(uintptr_t)ex.lists,
                                     (uint64_t)ex.list_cap, (uint64_t)limit, (uint64_t)ex.plane_cells,
                                     (uint64_t)(uintptr_t)ex.stream, (uint64_t)defer,
                                     (uint64_t)(uintptr_t)ex.item_slot,
                                     (uint64_t)P[idx[0]].n_periods, (uint64_t)ordered,
                                     (uint64_t)(uintptr_t)ex.order_keys, (uint64_t)max_periods};
        for (int k : idx) {
            key.push_back((uint64_t)(uintptr_t)plans[k].count);
            key.push_back((uint64_t)Ls[k]->ncells());
        }
        // fills + propagation; the events bracket this sequence (they are
        // recorded outside any graph capture)
        auto enqueue = [&]() -> hipError_t {
            hipError_t e = launch_fill_u32((uint32_t*)ex.rc, sizeof(RunCounters) / 4, 0u, ex.stream);
            if (e != hipSuccess) return e;
            if (defer) {
                e = launch_fill_u32((uint32_t*)ex.item_slot, (size_t)total * 2, 0xFFFFFFFFu, ex.stream);
                if (e != hipSuccess) return e;
            }
            for (int k : idx) {
                if (plans[k].count) {
                    e = launch_fill_u32(plans[k].count, (size_t)Ls[k]->ncells(), 0u, ex.stream);
                    if (e != hipSuccess) return e;
                }
            }
            if (ordered) {
                e = launch_order(precision, ex.d_jobs, (int)idx.size(), total, max_periods, ex.order_keys, ex.order,
                                 ex.stream);
                if (e != hipSuccess) return e;
            }
            e = launch_propagate(precision, lp.block, lp.grid, ex.d_jobs, (int)idx.size(), total, sl, ex.rc,
                                     ex.stream);
            if (e != hipSuccess || !defer) return e;
            return launch_dense_outputs(ex.d_jobs, (int)idx.size(), total, lp.grid, max_cells, sl, ex.rc,
                                        ex.stream);
        };
        bool launched = false;
        if (use_graph && !ex.graph_unavailable) {
            if (ex.graph_exec == nullptr || ex.graph_key != key) {
                drop_graph(ex);
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamBeginCapture(ex.stream, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    hipError_t e1 = enqueue();
                    hipError_t e2 = hipStreamEndCapture(ex.stream, &g);
                    e = (e1 != hipSuccess) ? e1 : e2;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&ex.graph_exec, g, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    if (g) (void)hipGraphDestroy(g);
                    ex.graph_exec = nullptr;
                    ex.graph_unavailable = true;
                } else {
                    ex.graph = g;
                    ex.graph_key = key;
                }
            }
            if (ex.graph_exec) {
                HIP_TRY(ctx, hipEventRecord(ex.ev0, ex.stream));
                HIP_TRY(ctx, hipGraphLaunch(ex.graph_exec, ex.stream));
                HIP_TRY(ctx, hipEventRecord(ex.ev1, ex.stream));
                launched = true;
            }
        }
        if (!launched) {
            HIP_TRY(ctx, hipEventRecord(ex.ev0, ex.stream));
            HIP_TRY(ctx, enqueue());
            HIP_TRY(ctx, hipEventRecord(ex.ev1, ex.stream));
        }
        HIP_TRY(ctx, hipMemcpyAsync(ex.rc_host, ex.rc, sizeof(RunCounters), hipMemcpyDeviceToHost, ex.stream));
        HIP_TRY(ctx, hipStreamSynchronize(ex.stream));
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ex.ev0, ex.ev1));
        ex.last.kernel_ms += ms;
        if (ex.rc_host->overflow == 0) {
            ex.last.entries += (int64_t)ex.rc_host->c[kCntEntries];
            ex.last.rate_evals += (int64_t)ex.rc_host->c[kCntEvals];
            ex.last.candidates += (int64_t)ex.rc_host->c[kCntCandidates];
            ex.last.improvements += (int64_t)ex.rc_host->c[kCntImprovements];
            ex.last.ignitions += (int64_t)ex.rc_host->c[kCntIgnitions];
            ex.last.rounds += (int64_t)ex.rc_host->c[kCntRounds];
            ex.last.continuations += (int64_t)ex.rc_host->c[kCntConts];
            ex.last.block_threads = lp.block;
            ex.last.grid_blocks = lp.grid;
            ex.last.list_capacity = limit;
            ex.last.rep_order = ordered ? 1 : 0;
            return C2F_OK;
        }
        ++ex.last.relaunches;
        const int64_t hard_max = std::min<int64_t>(std::max<int64_t>(4 * max_cells, 1 << 12) * 8, (int64_t)1 << 30);
        if (limit >= hard_max)
            return fail(ctx, C2F_ECAPACITY, "work lists overflow at capacity %lld", (long long)limit);
        lp.cap = std::min(hard_max, limit * 4);
        // remember the larger capacity for requests of this shape
        std::lock_guard<std::mutex> lk(ctx->tunemu);
        ctx->tune[TuneKey{max_cells, total, precision}] = TuneVal{lp.block, lp.cap};
    }
}

// Device bytes of the host-bound outputs of one request.
size_t host_output_bytes(const c2f_outputs& o, int64_t cells, int32_t reps) {
    if (o.on_device) return 0;
    const size_t n = (size_t)cells, r = (size_t)reps;
    auto sz = [](const void* p, size_t b) -> size_t { return p ? ((b + 255) & ~(size_t)255) : 0; };
    return sz(o.scar, r * n) + sz(o.arrival_period, r * n * 4) + sz(o.arrival_minute, r * n * 4) +
           sz(o.burn_count, n * 4) + sz(o.burned_cells, r * 8) + sz(o.ignition_cell, r * 4) +
           sz(o.scenario, r * 4);
}

// Run validated requests on one executor and deliver their outputs.
c2f_status run_requests(c2f_ctx* ctx, Exec& ex, const std::vector<c2f_sim_params>& P,
                        const std::vector<const Landscape*>& Ls, const std::vector<const Weather*>& Ws,
                        const c2f_outputs* outs, bool use_graph, int32_t grid_cap) {
    const int n_jobs = (int)P.size();
    int64_t total_items = 0;
    for (int k = 0; k < n_jobs; ++k) total_items += P[k].reps;
    if (total_items > 0x3FFFFFFF) return fail(ctx, C2F_EINVAL, "too many replications in one call");

    // plan outputs: device pointers directly, host ones through staging
    std::vector<OutPlan> plans(n_jobs);
    size_t stage = 0;
    auto need = [&](const void* want, size_t bytes) -> size_t {
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
    c2f_status st = ensure_staging(ctx, ex, stage);
    if (st != C2F_OK) return st;
    char* sb = (char*)ex.staging;
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

    memset(&ex.last, 0, sizeof ex.last);
    std::vector<int> g64, g32;
    for (int k = 0; k < n_jobs; ++k) (P[k].precision == 1 ? g32 : g64).push_back(k);
    if (!g64.empty() && !g32.empty()) use_graph = false;   // one cached graph per executor
    st = run_group(ctx, ex, g64, P, Ls, Ws, plans, 0, use_graph, grid_cap);
    if (st != C2F_OK) return st;
    st = run_group(ctx, ex, g32, P, Ls, Ws, plans, 1, use_graph, grid_cap);
    if (st != C2F_OK) return st;

    // copy host outputs back: the whole staging area in one transfer to
    // pinned memory, then each output to the caller's buffer
    if (stage > 0) {
        st = ensure_host_stage(ctx, ex, stage);
        if (st != C2F_OK) return st;
        HIP_TRY(ctx, hipMemcpyAsync(ex.host_stage, ex.staging, stage, hipMemcpyDeviceToHost, ex.stream));
    }
    HIP_TRY(ctx, hipStreamSynchronize(ex.stream));
    const char* hb = (const char*)ex.host_stage;
    for (int k = 0; k < n_jobs; ++k) {
        const c2f_outputs& o = outs[k];
        if (o.on_device) continue;
        const size_t n = (size_t)Ls[k]->ncells(), r = (size_t)P[k].reps;
        auto cp = [&](void* dst, size_t off, size_t bytes) {
            if (dst && off) memcpy(dst, hb + off - 1, bytes);
        };
        cp(o.scar, offs[k][0], r * n);
        cp(o.arrival_period, offs[k][1], r * n * 4);
        cp(o.arrival_minute, offs[k][2], r * n * 4);
        cp(o.burn_count, offs[k][3], n * 4);
        cp(o.burned_cells, offs[k][4], r * 8);
        cp(o.ignition_cell, offs[k][5], r * 4);
        cp(o.scenario, offs[k][6], r * 4);
    }
    return C2F_OK;
}

// Synchronous path: validate against the maps (caller holds ctx->mu), run
// on the main executor.
c2f_status simulate_impl(c2f_ctx* ctx, int32_t n_jobs, const c2f_sim_params* params, const c2f_outputs* outs,
                         bool use_graph) {
    if (n_jobs <= 0 || !params || !outs) return fail(ctx, C2F_EINVAL, "need n_jobs >= 1 and params/out arrays");
    std::vector<c2f_sim_params> P(params, params + n_jobs);
    std::vector<const Landscape*> Ls(n_jobs);
    std::vector<const Weather*> Ws(n_jobs);
    for (int k = 0; k < n_jobs; ++k) {
        Landscape* L;
        Weather* W;
        c2f_status st = check_params(ctx, &P[k], &L, &W);
        if (st != C2F_OK) return st;
        Ls[k] = L;
        Ws[k] = W;
    }
    return run_requests(ctx, ctx->main, P, Ls, Ws, outs, use_graph, 0);
}

// ---------------------------------------------------------------- serving

// Device bytes lane `ex` would add to run `batch`.
size_t batch_growth(c2f_ctx* ctx, const Exec& ex, const std::vector<std::shared_ptr<Ticket>>& batch) {
    int64_t cells[2] = {0, 0};
    int32_t items[2] = {0, 0};
    size_t stage = 0;
    for (const auto& t : batch) {
        const int pr = t->params.precision == 1 ? 1 : 0;
        cells[pr] = std::max(cells[pr], t->L->ncells());
        items[pr] += t->params.reps;
        stage += host_output_bytes(t->out, t->L->ncells(), t->params.reps);
    }
    int32_t grid = 1;
    int64_t cap = 1, max_cells = 1;
    for (int pr = 0; pr < 2; ++pr) {
        if (!items[pr]) continue;
        const LaunchPlan lp = plan_launch(ctx, cells[pr], items[pr], pr, ctx->max_batch_grid);
        grid = std::max(grid, std::min(lp.grid, lane_slot_cap(ctx->lane_plane_budget, cells[pr])));
        cap = std::max(cap, lp.cap);
        max_cells = std::max(max_cells, cells[pr]);
    }
    size_t g = exec_growth(ex, grid, max_cells, lane_list_cap(std::max(ctx->lane_list_budget, ex.list_pool), grid, cap), stage,
                           (int32_t)batch.size(), ctx->lane_plane_budget, ctx->lane_list_budget);
    const int32_t n_items = std::max(items[0], items[1]);
    if (n_items > grid && n_items > ex.order_cap)   // a launch in replication order
        g += ((size_t)pow2_at_least(std::max(n_items, 64)) - (size_t)ex.order_cap) * kOrderBytesPerItem;
    return g;
}

bool fits(c2f_ctx* ctx, size_t growth) {
    return bytes_in_use(ctx) + ctx->promised + growth <= ctx->admit_limit;
}

// Form the next batch for `ln` from the head of the queue (caller holds
// smu).  Requests are taken in arrival order while the lane's added device
// memory fits the admission limit; a head that does not fit waits for
// running lanes, and idle lanes give back their buffers to make room.
// Host-bound output bytes a batch collects before it stops taking requests
// (a single larger request still runs): keeps the lanes' staging buffers
// from growing, and each batch's results from waiting on a long transfer.
constexpr size_t kBatchHostBytes = (size_t)512 << 20;

bool try_admit(c2f_ctx* ctx, Lane& ln, std::vector<std::shared_ptr<Ticket>>& batch, size_t& growth) {
    batch.clear();
    growth = 0;
    if (ctx->queue.empty()) return false;
    int64_t items = 0;
    size_t host_bytes = 0;
    for (auto it = ctx->queue.begin(); it != ctx->queue.end(); ++it) {
        const auto& t = *it;
        if (!batch.empty() && items + t->params.reps > ctx->max_batch_reps) break;
        const size_t hb = host_output_bytes(t->out, t->L->ncells(), t->params.reps);
        if (!batch.empty() && host_bytes + hb > kBatchHostBytes) break;
        host_bytes += hb;
        batch.push_back(t);
        const size_t g = batch_growth(ctx, ln.ex, batch);
        if (!fits(ctx, g)) {
            batch.pop_back();
            break;
        }
        growth = g;
        items += t->params.reps;
    }
    if (batch.empty()) {
        // make room: idle lanes release their buffers
        for (auto& other : ctx->lanes)
            if (other.get() != &ln && !other->busy) exec_trim(ctx, other->ex);
        batch.push_back(ctx->queue.front());
        size_t g = batch_growth(ctx, ln.ex, batch);
        if (!fits(ctx, g)) {
            if (ctx->busy_lanes > 0) {
                batch.clear();
                return false;   // wait for running batches to finish
            }
            // alone on the device: start from empty buffers and let the
            // launch shrink its grid if memory is short
            exec_trim(ctx, ln.ex);
            g = batch_growth(ctx, ln.ex, batch);
        }
        growth = g;
    }
    ctx->queue.erase(ctx->queue.begin(), ctx->queue.begin() + (ptrdiff_t)batch.size());
    return true;
}

void lane_loop(c2f_ctx* ctx, Lane* ln) {
    (void)hipSetDevice(ctx->device);
    for (;;) {
        std::vector<std::shared_ptr<Ticket>> batch;
        size_t growth = 0;
        {
            std::unique_lock<std::mutex> lk(ctx->smu);
            for (;;) {
                if (ctx->stopping && ctx->queue.empty()) return;
                if (try_admit(ctx, *ln, batch, growth)) break;
                ctx->scv.wait(lk);
            }
            ln->busy = true;
            ++ctx->busy_lanes;
            ctx->promised += growth;
        }
        const double t_start = ms_since(ctx->t0);
        int32_t items = 0;
        std::vector<c2f_sim_params> P;
        std::vector<const Landscape*> Ls;
        std::vector<const Weather*> Ws;
        std::vector<c2f_outputs> O;
        for (auto& t : batch) {
            P.push_back(t->params);
            Ls.push_back(t->L);
            Ws.push_back(t->W);
            O.push_back(t->out);
            items += t->params.reps;
        }
        t_err.clear();
        clear_sticky_error();
        std::vector<c2f_status> st(batch.size());
        std::vector<std::string> err(batch.size());
        std::vector<double> kms(batch.size());
        c2f_status s0 = run_requests(ctx, ln->ex, P, Ls, Ws, O.data(), false, ctx->max_batch_grid);
        if (s0 == C2F_OK || batch.size() == 1) {
            for (size_t k = 0; k < batch.size(); ++k) {
                st[k] = s0;
                err[k] = t_err;
                kms[k] = ln->ex.last.kernel_ms;
            }
        } else {
            // run one by one so that a failing request only fails itself
            for (size_t k = 0; k < batch.size(); ++k) {
                t_err.clear();
                clear_sticky_error();
                std::vector<c2f_sim_params> P1{P[k]};
                std::vector<const Landscape*> L1{Ls[k]};
                std::vector<const Weather*> W1{Ws[k]};
                st[k] = run_requests(ctx, ln->ex, P1, L1, W1, &O[k], false, ctx->max_batch_grid);
                err[k] = t_err;
                kms[k] = ln->ex.last.kernel_ms;
            }
        }
        const double t_done = ms_since(ctx->t0);
        {
            std::lock_guard<std::mutex> lk(ctx->objmu);
            for (auto& t : batch) {
                --t->L->inflight;
                --t->W->inflight;
            }
        }
        {
            std::lock_guard<std::mutex> lk(ctx->smu);
            ctx->promised -= std::min(ctx->promised, growth);
            ln->busy = false;
            --ctx->busy_lanes;
            for (size_t k = 0; k < batch.size(); ++k) {
                Ticket& t = *batch[k];
                t.status = st[k];
                t.err = err[k];
                t.info.start_ms = t_start;
                t.info.done_ms = t_done;
                t.info.kernel_ms = kms[k];
                t.info.batch_requests = (int32_t)batch.size();
                t.info.batch_reps = items;
                t.info.lane = ln->index;
                t.info.status = st[k];
                t.done = true;
            }
        }
        ctx->scv.notify_all();
    }
}

// A lane's long-lived buffers, taken when serving starts rather than in
// the middle of a stream, where an allocation of many GB stalls for a
// second and a free waits for the whole device: the plane pool, and
// output staging (device and pinned host) for a batch's host-bound
// outputs, each within the lane's share of the serving memory.
c2f_status lane_reserve(c2f_ctx* ctx, Exec& ex) {
    const size_t budget = ctx->lane_plane_budget;
    if (budget >= ((size_t)64 << 20) && !ex.planes) {
        c2f_status st = dev_alloc(ctx, (void**)&ex.planes, budget);
        if (st != C2F_OK) return st;
        ex.plane_pool = budget;
        ex.plane_cells = 0;
        ex.tag_ready = 0;
    }
    if (ctx->lane_list_budget >= ((size_t)16 << 20) && !ex.lists) {
        c2f_status st = dev_alloc(ctx, (void**)&ex.lists, ctx->lane_list_budget);
        if (st != C2F_OK) return st;
        ex.list_pool = ctx->lane_list_budget;
        ex.list_cap = 0;
        ex.list_slots = 0;
    }
    const size_t stage = std::min(kBatchHostBytes, budget / 8);
    if (stage >= ((size_t)1 << 20)) {
        c2f_status st = ensure_staging(ctx, ex, stage);
        if (st == C2F_OK) st = ensure_host_stage(ctx, ex, stage);
        if (st != C2F_OK) return st;
    }
    return C2F_OK;
}

// Start the serving lanes (caller holds smu).
c2f_status start_lanes(c2f_ctx* ctx) {
    if (!ctx->lanes.empty()) return C2F_OK;
    // each lane's pools: a share of the admission memory left beside the
    // resident inputs (half of it split over the lanes, at most 20 GiB),
    // three quarters for planes and one for lists
    {
        const size_t held = bytes_in_use(ctx);
        const size_t avail = ctx->admit_limit > held ? (size_t)ctx->admit_limit - held : 0;
        const size_t share = std::min<size_t>((size_t)20 << 30, avail / (2 * (size_t)std::max(1, ctx->n_lanes)));
        ctx->lane_plane_budget = share / 4 * 3;
        ctx->lane_list_budget = share / 4;
    }
    for (int32_t i = 0; i < ctx->n_lanes; ++i) {
        std::unique_ptr<Lane> ln(new Lane());
        ln->index = i;
        c2f_status st = exec_init(ctx, ln->ex, true);
        if (st == C2F_OK) st = lane_reserve(ctx, ln->ex);
        if (st != C2F_OK) {
            exec_release(ctx, ln->ex);
            for (auto& l : ctx->lanes) exec_release(ctx, l->ex);
            ctx->lanes.clear();
            return st;
        }
        ctx->lanes.push_back(std::move(ln));
    }
    for (auto& ln : ctx->lanes) ln->th = std::thread(lane_loop, ctx, ln.get());
    return C2F_OK;
}

}  // namespace

// ===================================================================== ABI

// Launch sizes of a no-allocation run: everything inside the device scratch.
namespace {
constexpr int64_t kNoallocFirstCap = 4096;   // list entries per slot before any overflow

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

void record_stats(Exec& ex, const RunCounters& rc, int32_t block, int32_t grid, int64_t cap, float ms) {
    ex.last.kernel_ms += ms;
    ex.last.entries += (int64_t)rc.c[kCntEntries];
    ex.last.rate_evals += (int64_t)rc.c[kCntEvals];
    ex.last.candidates += (int64_t)rc.c[kCntCandidates];
    ex.last.improvements += (int64_t)rc.c[kCntImprovements];
    ex.last.ignitions += (int64_t)rc.c[kCntIgnitions];
    ex.last.rounds += (int64_t)rc.c[kCntRounds];
    ex.last.continuations += (int64_t)rc.c[kCntConts];
    ex.last.block_threads = block;
    ex.last.grid_blocks = grid;
    ex.last.list_capacity = cap;
    ex.last.rep_order = 0;
}
}  // namespace

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
    ctx->t0 = std::chrono::steady_clock::now();
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return C2F_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return C2F_EDEVICE;
    ctx->n_cu = prop.multiProcessorCount;
    ctx->arch.assign(prop.gcnArchName, strcspn(prop.gcnArchName, ": \t\n"));
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return C2F_EDEVICE;
    ctx->admit_limit = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
    // the no-allocation scratch: its address on this device, resolved once
    // per device with the device current
    if (scratch_resolve(device, &ctx->scratch) != hipSuccess) {
        (void)hipGetLastError();
        return C2F_EDEVICE;
    }
    if (exec_init(ctx.get(), ctx->main, false) != C2F_OK) {
        exec_release(ctx.get(), ctx->main);
        return C2F_EDEVICE;
    }
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
    for (auto& ln : ctx->lanes)
        if (ln->th.joinable()) ln->th.join();
    (void)hipSetDevice(ctx->device);
    for (auto& ln : ctx->lanes) exec_release(ctx, ln->ex);
    ctx->lanes.clear();
    exec_release(ctx, ctx->main);
    if (ctx->metric_buf) (void)hipFree(ctx->metric_buf);
    if (ctx->acct) (void)hipFree(ctx->acct);
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
    delete ctx;
}

const char* c2f_last_error(const c2f_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

c2f_status c2f_set_stream(c2f_ctx* ctx, void* hip_stream) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    drop_graph(ctx->main);
    ctx->main.stream = hip_stream ? (hipStream_t)hip_stream : ctx->main.own_stream;
    return C2F_OK;
}

c2f_status c2f_load_landscape(c2f_ctx* ctx, int32_t rows, int32_t cols, int32_t cell_m, const uint8_t* fuel,
                              const int16_t* elev_m, float pc_pct, float curing_pct, int32_t* landscape_id) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (rows <= 0 || cols <= 0 || (int64_t)rows * cols > 0x7FFFFFFEll)
        return fail(ctx, C2F_EINVAL, "grid %d x %d out of range", rows, cols);
    if (cell_m < 1 || cell_m > 20000) return fail(ctx, C2F_EINVAL, "cell_m %d not in 1..20000", cell_m);
    if (!fuel || !landscape_id) return fail(ctx, C2F_EINVAL, "fuel and landscape_id must be non-NULL");
    if (!(pc_pct >= 0.f && pc_pct <= 100.f)) return fail(ctx, C2F_EINVAL, "pc_pct must be in 0..100");
    if (!(curing_pct > 0.f && curing_pct <= 100.f)) return fail(ctx, C2F_EINVAL, "curing_pct must be in (0, 100]");
    const int64_t n = (int64_t)rows * cols;
    for (int64_t i = 0; i < n; ++i)
        if (fuel[i] >= kNumFuels)
            return fail(ctx, C2F_EINVAL, "fuel code %d at cell %lld > %d", fuel[i], (long long)i, kNumFuels - 1);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->main.stream;
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
    hipError_t e = hipMemcpyAsync(L.fuel, fuel, (size_t)n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && elev_m) e = hipMemcpyAsync(d_elev, elev_m, (size_t)n * 2, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_prepare_landscape(L.fuel, d_elev, nullptr, rows, cols, cell_m, pc_pct, curing_pct, L.fmc, L.pdf,
                                     L.cells, L.burnable, d_tiles, L.land, s);
    LandDev hl;
    if (e == hipSuccess) e = hipMemcpyAsync(&hl, L.land, sizeof hl, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
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
    std::lock_guard<std::mutex> lk2(ctx->objmu);
    const int32_t id = ctx->next_id++;
    ctx->lands[id] = L;
    *landscape_id = id;
    return C2F_OK;
}

c2f_status c2f_derive_landscape(c2f_ctx* ctx, int32_t base_id, int64_t n_edits, const int32_t* cells,
                                const uint8_t* fuels, int32_t* landscape_id) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!landscape_id) return fail(ctx, C2F_EINVAL, "landscape_id must be non-NULL");
    if (n_edits < 0 || (n_edits > 0 && (!cells || !fuels)))
        return fail(ctx, C2F_EINVAL, "need n_edits >= 0 and non-NULL cells/fuels");
    Landscape B;
    {
        std::lock_guard<std::mutex> lk2(ctx->objmu);
        auto it = ctx->lands.find(base_id);
        if (it == ctx->lands.end()) return fail(ctx, C2F_ESTATE, "unknown landscape id %d", base_id);
        B = it->second;
    }
    const int64_t n = B.ncells();
    for (int64_t k = 0; k < n_edits; ++k) {
        if (cells[k] < 0 || cells[k] >= n)
            return fail(ctx, C2F_EINVAL, "edit %lld: cell %d outside the grid", (long long)k, cells[k]);
        if (fuels[k] >= kNumFuels)
            return fail(ctx, C2F_EINVAL, "edit %lld: fuel code %d > %d", (long long)k, fuels[k], kNumFuels - 1);
    }
    // one edit per cell, the last one given (the device applies them in parallel)
    std::vector<int64_t> order((size_t)n_edits);
    for (int64_t k = 0; k < n_edits; ++k) order[(size_t)k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cells[a] < cells[b]; });
    std::vector<int32_t> ucells;
    std::vector<uint8_t> ucodes;
    for (size_t i = 0; i < order.size(); ++i) {
        if (i + 1 < order.size() && cells[order[i + 1]] == cells[order[i]]) continue;
        ucells.push_back(cells[order[i]]);
        ucodes.push_back(fuels[order[i]]);
    }
    n_edits = (int64_t)ucells.size();
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->main.stream;
    Landscape L;
    L.rows = B.rows;
    L.cols = B.cols;
    L.cell_m = B.cell_m;
    L.pc = B.pc;
    L.curing = B.curing;
    L.fmc = B.fmc;
    L.pdf = B.pdf;
    int32_t* d_tiles = nullptr;
    int32_t* d_cells = nullptr;
    uint8_t* d_codes = nullptr;
    const int64_t n_tiles = tile_scratch_entries(n);
    const size_t ne = (size_t)std::max<int64_t>(n_edits, 1);
    auto temps = [&]() {
        dev_free(ctx, d_tiles, (size_t)n_tiles * 4);
        dev_free(ctx, d_cells, ne * 4);
        dev_free(ctx, d_codes, ne);
        d_tiles = nullptr;
        d_cells = nullptr;
        d_codes = nullptr;
    };
    auto cleanup = [&]() {
        temps();
        dev_free(ctx, L.fuel, (size_t)n);
        dev_free(ctx, L.cells, (size_t)n * sizeof(CellRec));
        dev_free(ctx, L.burnable, (size_t)n * 4);
        dev_free(ctx, L.land, sizeof(LandDev));
    };
    c2f_status st = C2F_OK;
    if ((st = dev_alloc(ctx, (void**)&L.fuel, (size_t)n)) != C2F_OK ||
        (st = dev_alloc(ctx, (void**)&L.cells, (size_t)n * sizeof(CellRec))) != C2F_OK ||
        (st = dev_alloc(ctx, (void**)&L.burnable, (size_t)n * 4)) != C2F_OK ||
        (st = dev_alloc(ctx, (void**)&L.land, sizeof(LandDev))) != C2F_OK ||
        (st = dev_alloc(ctx, (void**)&d_tiles, (size_t)n_tiles * 4)) != C2F_OK ||
        (st = dev_alloc(ctx, (void**)&d_cells, ne * 4)) != C2F_OK ||
        (st = dev_alloc(ctx, (void**)&d_codes, ne)) != C2F_OK) {
        cleanup();
        return st;
    }
    // the base's fuel with the edits applied; slopes from the base's records
    hipError_t e = hipMemcpyAsync(L.fuel, B.fuel, (size_t)n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && n_edits > 0)
        e = hipMemcpyAsync(d_cells, ucells.data(), (size_t)n_edits * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n_edits > 0)
        e = hipMemcpyAsync(d_codes, ucodes.data(), (size_t)n_edits, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_fuel_edits(L.fuel, d_cells, d_codes, n_edits, s);
    if (e == hipSuccess)
        e = launch_prepare_landscape(L.fuel, nullptr, B.cells, L.rows, L.cols, L.cell_m, L.pc, L.curing, L.fmc,
                                     L.pdf, L.cells, L.burnable, d_tiles, L.land, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    temps();
    if (e != hipSuccess) {
        cleanup();
        return fail(ctx, C2F_EDEVICE, "derived landscape preparation failed: %s", hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> lk2(ctx->objmu);
    const int32_t id = ctx->next_id++;
    ctx->lands[id] = L;
    *landscape_id = id;
    return C2F_OK;
}

c2f_status c2f_unload_landscape(c2f_ctx* ctx, int32_t landscape_id) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Landscape L;
    {
        std::lock_guard<std::mutex> lk2(ctx->objmu);
        auto it = ctx->lands.find(landscape_id);
        if (it == ctx->lands.end()) return fail(ctx, C2F_ESTATE, "unknown landscape id %d", landscape_id);
        if (it->second.inflight > 0)
            return fail(ctx, C2F_EBUSY, "landscape %d is used by %d submitted requests", landscape_id,
                        it->second.inflight);
        L = it->second;
        ctx->lands.erase(it);
    }
    (void)hipStreamSynchronize(ctx->main.stream);
    drop_graph(ctx->main);
    const size_t n = (size_t)L.ncells();
    dev_free(ctx, L.fuel, n);
    dev_free(ctx, L.cells, n * sizeof(CellRec));
    dev_free(ctx, L.burnable, n * 4);
    dev_free(ctx, L.land, sizeof(LandDev));
    dev_free(ctx, L.ign_cdf, n * 8);
    return C2F_OK;
}

namespace {
// Shared checks of the scar comparison entry points.
c2f_status check_scar_args(c2f_ctx* ctx, int64_t n_cells, int32_t n_periods, int32_t period_min,
                           const void* arrival_minute, const void* reference) {
    if (n_cells < 2 || n_cells > 0x7FFFFFFEll) return fail(ctx, C2F_EINVAL, "n_cells must be in 2..2^31-2");
    if (n_periods < 1 || n_periods > 65535) return fail(ctx, C2F_EINVAL, "n_periods must be in 1..65535");
    if (period_min < 1) return fail(ctx, C2F_EINVAL, "period_min must be >= 1");
    if (!arrival_minute || !reference) return fail(ctx, C2F_EINVAL, "arrival_minute and reference must be non-NULL");
    return C2F_OK;
}

// The context's scar comparison buffer, laid out for its capacity C >= T
// periods: counts (3 C u64) and the ticket of the last finishing block, both
// zero between launches (a launch clears what it used), then 2 C + 1 f64
// results.  The layout depends on C only, so results never land where a
// later launch's counts must be zero.  Grown on demand (work queued on s
// before a regrowth is waited for; a new buffer is zeroed on s).  Needs
// ctx->mu.
c2f_status scar_buffers(c2f_ctx* ctx, size_t T, hipStream_t s, unsigned long long** cnt, uint32_t** ticket,
                        double** out) {
    if (ctx->metric_periods < T) {
        const size_t C = T;
        const size_t need = ((C * 24 + 255) & ~(size_t)255) + 256 + (2 * C + 1) * 8;
        if (ctx->metric_buf) {
            HIP_TRY(ctx, hipStreamSynchronize(s));
            dev_free(ctx, ctx->metric_buf, ctx->metric_bytes);
            ctx->metric_buf = nullptr;
            ctx->metric_bytes = 0;
            ctx->metric_periods = 0;
        }
        const c2f_status st = dev_alloc(ctx, &ctx->metric_buf, need);
        if (st != C2F_OK) return st;
        ctx->metric_bytes = need;
        const size_t zero_bytes = ((C * 24 + 255) & ~(size_t)255) + 256;
        const hipError_t e = launch_fill_u32((uint32_t*)ctx->metric_buf, zero_bytes / 4, 0u, s);
        if (e != hipSuccess) {
            dev_free(ctx, ctx->metric_buf, ctx->metric_bytes);
            ctx->metric_buf = nullptr;
            ctx->metric_bytes = 0;
            return fail(ctx, C2F_EDEVICE, "clearing the scar count buffer failed: %s", hipGetErrorString(e));
        }
        ctx->metric_periods = C;
    }
    const size_t cnt_bytes = (ctx->metric_periods * 24 + 255) & ~(size_t)255;
    *cnt = (unsigned long long*)ctx->metric_buf;
    *ticket = (uint32_t*)((char*)ctx->metric_buf + cnt_bytes);
    *out = (double*)((char*)ctx->metric_buf + cnt_bytes + 256);
    return C2F_OK;
}
}  // namespace

c2f_status c2f_compare_scars(c2f_ctx* ctx, int64_t n_cells, int32_t n_periods, int32_t period_min,
                             const int32_t* arrival_minute, const uint8_t* reference, int32_t on_device,
                             double* mse, double* ssim, double* delta_norm) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    c2f_status st = check_scar_args(ctx, n_cells, n_periods, period_min, arrival_minute, reference);
    if (st != C2F_OK) return st;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->main.stream;
    const size_t n = (size_t)n_cells, T = (size_t)n_periods;
    unsigned long long* d_cnt = nullptr;
    uint32_t* d_ticket = nullptr;
    double* d_out = nullptr;
    if ((st = scar_buffers(ctx, T, s, &d_cnt, &d_ticket, &d_out)) != C2F_OK) return st;
    int32_t* d_arr = nullptr;
    uint8_t* d_ref = nullptr;
    auto cleanup = [&]() {
        if (!on_device) {
            dev_free(ctx, d_arr, n * 4);
            dev_free(ctx, d_ref, n * T);
        }
    };
    if (on_device) {
        d_arr = const_cast<int32_t*>(arrival_minute);
        d_ref = const_cast<uint8_t*>(reference);
    } else if ((st = dev_alloc(ctx, (void**)&d_arr, n * 4)) != C2F_OK ||
               (st = dev_alloc(ctx, (void**)&d_ref, n * T)) != C2F_OK) {
        cleanup();
        return st;
    }
    hipError_t e = hipSuccess;
    if (!on_device) {
        e = hipMemcpyAsync(d_arr, arrival_minute, n * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_ref, reference, n * T, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess)
        e = launch_scar_metrics(d_arr, d_ref, n_cells, n_periods, period_min, d_cnt, d_ticket, d_out, s);
    std::vector<double> out(2 * T + 1);
    if (e == hipSuccess) e = hipMemcpyAsync(out.data(), d_out, out.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) return fail(ctx, C2F_EDEVICE, "scar comparison failed: %s", hipGetErrorString(e));
    if (mse) std::copy(out.begin(), out.begin() + (ptrdiff_t)T, mse);
    if (ssim) std::copy(out.begin() + (ptrdiff_t)T, out.begin() + (ptrdiff_t)(2 * T), ssim);
    if (delta_norm) *delta_norm = out[2 * T];
    return C2F_OK;
}

c2f_status c2f_compare_scars_async(c2f_ctx* ctx, int64_t n_cells, int32_t n_periods, int32_t period_min,
                                   const int32_t* arrival_minute, const uint8_t* reference, double* results) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    c2f_status st = check_scar_args(ctx, n_cells, n_periods, period_min, arrival_minute, reference);
    if (st != C2F_OK) return st;
    if (!results) return fail(ctx, C2F_EINVAL, "results must be non-NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->main.stream;
    const size_t T = (size_t)n_periods;
    unsigned long long* d_cnt = nullptr;
    uint32_t* d_ticket = nullptr;
    double* d_out = nullptr;
    if ((st = scar_buffers(ctx, T, s, &d_cnt, &d_ticket, &d_out)) != C2F_OK) return st;
    hipError_t e =
        launch_scar_metrics(arrival_minute, reference, n_cells, n_periods, period_min, d_cnt, d_ticket, results, s);
    if (e != hipSuccess) return fail(ctx, C2F_EDEVICE, "scar comparison failed: %s", hipGetErrorString(e));
    return C2F_OK;
}

c2f_status c2f_set_ignition_map(c2f_ctx* ctx, int32_t landscape_id, const uint32_t* weights) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    std::lock_guard<std::mutex> lk2(ctx->objmu);
    auto it = ctx->lands.find(landscape_id);
    if (it == ctx->lands.end()) return fail(ctx, C2F_ESTATE, "unknown landscape id %d", landscape_id);
    Landscape& L = it->second;
    if (L.inflight > 0)
        return fail(ctx, C2F_EBUSY, "landscape %d is used by %d submitted requests", landscape_id, L.inflight);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const size_t n = (size_t)L.ncells();
    if (L.ign_cdf) {
        (void)hipStreamSynchronize(ctx->main.stream);
        drop_graph(ctx->main);
        dev_free(ctx, L.ign_cdf, n * 8);
        L.ign_cdf = nullptr;
        L.ign_total = 0;
    }
    if (!weights) return C2F_OK;
    // running sums in 64 bits: at most 2^31 cells of weight below 2^32
    std::vector<uint64_t> cdf(n);
    uint64_t run = 0;
    for (size_t i = 0; i < n; ++i) {
        run += weights[i];
        cdf[i] = run;
    }
    uint64_t* d = nullptr;
    c2f_status st = dev_alloc(ctx, (void**)&d, n * 8);
    if (st != C2F_OK) return st;
    if (hipMemcpy(d, cdf.data(), n * 8, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        dev_free(ctx, d, n * 8);
        return fail(ctx, C2F_EDEVICE, "ignition map upload failed");
    }
    L.ign_cdf = d;
    L.ign_total = run;
    return C2F_OK;
}

c2f_status c2f_set_weather(c2f_ctx* ctx, int32_t n_scen, int32_t n_periods, int32_t period_min,
                           const c2f_weather_row* rows, int32_t* weather_id) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
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
    hipStream_t s = ctx->main.stream;
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
    hipError_t e = hipMemcpyAsync(W.rows, rows, (size_t)nr * 16, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_weather_table(W.rows, (int)nr, W.t64, W.t32, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        dev_free(ctx, W.rows, (size_t)nr * 16);
        dev_free(ctx, W.t64, (size_t)nr * kRowLen * 8);
        dev_free(ctx, W.t32, (size_t)nr * kRowLen * 4);
        return fail(ctx, C2F_EDEVICE, "weather upload failed: %s", hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> lk2(ctx->objmu);
    const int32_t id = ctx->next_id++;
    ctx->weathers[id] = W;
    *weather_id = id;
    return C2F_OK;
}

c2f_status c2f_unset_weather(c2f_ctx* ctx, int32_t weather_id) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Weather W;
    {
        std::lock_guard<std::mutex> lk2(ctx->objmu);
        auto it = ctx->weathers.find(weather_id);
        if (it == ctx->weathers.end()) return fail(ctx, C2F_ESTATE, "unknown weather id %d", weather_id);
        if (it->second.inflight > 0)
            return fail(ctx, C2F_EBUSY, "weather %d is used by %d submitted requests", weather_id,
                        it->second.inflight);
        W = it->second;
        ctx->weathers.erase(it);
    }
    (void)hipStreamSynchronize(ctx->main.stream);
    drop_graph(ctx->main);
    const size_t nr = (size_t)W.n_scen * W.n_periods;
    dev_free(ctx, W.rows, nr * 16);
    dev_free(ctx, W.t64, nr * kRowLen * 8);
    dev_free(ctx, W.t32, nr * kRowLen * 4);
    return C2F_OK;
}

c2f_status c2f_simulate(c2f_ctx* ctx, const c2f_sim_params* params, const c2f_outputs* out) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, C2F_EDEVICE, "hipSetDevice failed");
    return simulate_impl(ctx, 1, params, out, true);
}

c2f_status c2f_simulate_batch(c2f_ctx* ctx, int32_t n_jobs, const c2f_sim_params* params, const c2f_outputs* out) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, C2F_EDEVICE, "hipSetDevice failed");
    return simulate_impl(ctx, n_jobs, params, out, true);
}

c2f_status c2f_simulate_noalloc(c2f_ctx* ctx, const c2f_sim_params* params, const c2f_outputs* out) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, C2F_EDEVICE, "hipSetDevice failed");
    if (!out) return fail(ctx, C2F_EINVAL, "out is NULL");
    if (!out->on_device) return fail(ctx, C2F_EINVAL, "c2f_simulate_noalloc needs device outputs (on_device = 1)");
    if (!ctx->scratch) return fail(ctx, C2F_EDEVICE, "no device scratch on device %d", ctx->device);
    Landscape* L;
    Weather* W;
    c2f_status st = check_params(ctx, params, &L, &W);
    if (st != C2F_OK) return st;
    const c2f_sim_params& p = *params;
    const int64_t cells = L->ncells();
    OutPlan o;
    o.user = *out;
    o.scar = out->scar;
    o.arr_period = out->arrival_period;
    o.arr_minute = out->arrival_minute;
    o.count = out->burn_count;
    o.burned = out->burned_cells;
    o.ign = out->ignition_cell;
    o.scen = out->scenario;
    LaunchPlan lp = plan_launch(ctx, cells, p.reps, p.precision, 0);
    // Layout: run counters | job record | tags[slots] | planes[slots] | lists[slots]
    const size_t head = align256(sizeof(RunCounters)) + align256(sizeof(Job));
    const size_t plane_b = align256((size_t)cells * 4);
    const int64_t cap_max = std::min<int64_t>(std::max<int64_t>(4 * cells, 1 << 12) * 8, (int64_t)1 << 30);
    int64_t cap = std::min<int64_t>(std::min(lp.cap, kNoallocFirstCap), cap_max);
    Exec& ex = ctx->main;
    std::lock_guard<std::mutex> slk(scratch_lock(ctx->device));
    uint8_t* const base = (uint8_t*)ctx->scratch;
    RunCounters* const rc = (RunCounters*)base;
    Job* const job = (Job*)(base + align256(sizeof(RunCounters)));
    memset(&ex.last, 0, sizeof ex.last);
    for (;;) {
        const size_t per_slot = plane_b + (size_t)cap * kSlotListBytesPerEntry + 4;
        const size_t avail = kScratchBytes - head - 256;   // 256: the tag array's rounding
        const int64_t fit = (int64_t)(avail / per_slot);
        if (fit < 1)
            return fail(ctx, C2F_EINVAL,
                        "request needs %zu bytes of device scratch for one work slot (%lld cells, %lld list "
                        "entries); c2f_simulate_noalloc has %zu bytes (use c2f_simulate)",
                        head + 256 + per_slot, (long long)cells, (long long)cap, kScratchBytes);
        const int32_t slots = (int32_t)std::min<int64_t>(lp.grid, fit);
        uint32_t* const tags = (uint32_t*)(base + head);
        uint32_t* const planes = (uint32_t*)(base + head + align256((size_t)slots * 4));
        uint8_t* const lists = (uint8_t*)planes + (size_t)slots * plane_b;
        if (lists + (size_t)slots * (size_t)cap * kSlotListBytesPerEntry > base + kScratchBytes)
            return fail(ctx, C2F_EINVAL, "scratch layout exceeds the scratch");   // cannot happen
        const Slots sl{planes, (int64_t)(plane_b / 4), lists, cap, cap, tags, nullptr, nullptr};
        // tags 0: every slot refills its plane before its first replication,
        // so nothing a previous call left in the scratch is read
        HIP_TRY(ctx, launch_fill_u32((uint32_t*)rc, sizeof(RunCounters) / 4, 0u, ex.stream));
        HIP_TRY(ctx, launch_fill_u32(tags, (size_t)slots, 0u, ex.stream));
        if (o.count) HIP_TRY(ctx, launch_fill_u32(o.count, (size_t)cells, 0u, ex.stream));
        HIP_TRY(ctx, launch_store_job(make_job(p, *L, *W, o, p.precision, 0), job, ex.stream));
        HIP_TRY(ctx, hipEventRecord(ex.ev0, ex.stream));
        HIP_TRY(ctx, launch_propagate(p.precision, lp.block, slots, job, 1, p.reps, sl, rc, ex.stream));
        HIP_TRY(ctx, hipEventRecord(ex.ev1, ex.stream));
        HIP_TRY(ctx, hipMemcpyAsync(ex.rc_host, rc, sizeof(RunCounters), hipMemcpyDeviceToHost, ex.stream));
        HIP_TRY(ctx, hipStreamSynchronize(ex.stream));
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ex.ev0, ex.ev1));
        if (ex.rc_host->overflow == 0) {
            record_stats(ex, *ex.rc_host, lp.block, slots, cap, ms);
            return C2F_OK;
        }
        ++ex.last.relaunches;
        if (cap >= cap_max)
            return fail(ctx, C2F_ECAPACITY, "work lists overflow at capacity %lld", (long long)cap);
        cap = std::min(cap_max, cap * 4);
    }
}

c2f_status c2f_count_work(c2f_ctx* ctx, const c2f_sim_params* params, const int32_t* arrival_minute,
                          int64_t* counts) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, C2F_EDEVICE, "hipSetDevice failed");
    if (!arrival_minute || !counts) return fail(ctx, C2F_EINVAL, "arrival_minute and counts are required");
    Landscape* L;
    Weather* W;
    c2f_status st = check_params(ctx, params, &L, &W);
    if (st != C2F_OK) return st;
    const size_t job_off = 256;
    if (!ctx->acct) {
        st = dev_alloc(ctx, &ctx->acct, job_off + sizeof(Job));
        if (st != C2F_OK) return st;
    }
    Exec& ex = ctx->main;
    unsigned long long* cnt = (unsigned long long*)ctx->acct;
    Job* job = (Job*)((char*)ctx->acct + job_off);
    const OutPlan none;
    HIP_TRY(ctx, launch_fill_u32((uint32_t*)cnt, 6, 0u, ex.stream));
    HIP_TRY(ctx, launch_store_job(make_job(*params, *L, *W, none, params->precision, 0), job, ex.stream));
    HIP_TRY(ctx, launch_work_counts(params->precision, job, L->ncells() * (int64_t)params->reps, arrival_minute,
                                    cnt, ex.stream));
    unsigned long long h[3];
    HIP_TRY(ctx, hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, ex.stream));
    HIP_TRY(ctx, hipStreamSynchronize(ex.stream));
    for (int k = 0; k < 3; ++k) counts[k] = (int64_t)h[k];
    return C2F_OK;
}

c2f_status c2f_eval_ros(c2f_ctx* ctx, int32_t landscape_id, int32_t weather_id, int32_t scenario, int32_t period,
                        int32_t rep, uint64_t seed, float sigma, int32_t rounding, int32_t precision, double* hros,
                        double* bros, double* fros, double* lb, double* raz_deg, double* x8, int32_t* q8,
                        double* cfb, double* hfi) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
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
    Exec& ex = ctx->main;
    const size_t n = (size_t)L.ncells();
    const size_t bytes = n * 8 * 7 + n * 64 + n * 32 + 9 * 256;   // 9 arrays, 256-byte aligned
    c2f_status st = ensure_staging(ctx, ex, bytes);
    if (st != C2F_OK) return st;
    char* sb = (char*)ex.staging;
    EvalArgs a;
    memset(&a, 0, sizeof a);
    a.cells = L.cells;
    a.land = L.land;
    a.table = precision == 1 ? (const void*)W.t32 : (const void*)W.t64;
    a.table64 = W.t64;
    a.table32 = W.t32;
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
    a.cfb = cfb ? (double*)take(n * 8) : nullptr;
    a.hfi = hfi ? (double*)take(n * 8) : nullptr;
    HIP_TRY(ctx, launch_eval_ros(precision, a, ex.stream));
    if (hros) HIP_TRY(ctx, hipMemcpyAsync(hros, a.hros, n * 8, hipMemcpyDeviceToHost, ex.stream));
    if (bros) HIP_TRY(ctx, hipMemcpyAsync(bros, a.bros, n * 8, hipMemcpyDeviceToHost, ex.stream));
    if (fros) HIP_TRY(ctx, hipMemcpyAsync(fros, a.fros, n * 8, hipMemcpyDeviceToHost, ex.stream));
    if (lb) HIP_TRY(ctx, hipMemcpyAsync(lb, a.lb, n * 8, hipMemcpyDeviceToHost, ex.stream));
    if (raz_deg) HIP_TRY(ctx, hipMemcpyAsync(raz_deg, a.raz, n * 8, hipMemcpyDeviceToHost, ex.stream));
    if (x8) HIP_TRY(ctx, hipMemcpyAsync(x8, a.x8, n * 64, hipMemcpyDeviceToHost, ex.stream));
    if (q8) HIP_TRY(ctx, hipMemcpyAsync(q8, a.q8, n * 32, hipMemcpyDeviceToHost, ex.stream));
    if (cfb) HIP_TRY(ctx, hipMemcpyAsync(cfb, a.cfb, n * 8, hipMemcpyDeviceToHost, ex.stream));
    if (hfi) HIP_TRY(ctx, hipMemcpyAsync(hfi, a.hfi, n * 8, hipMemcpyDeviceToHost, ex.stream));
    HIP_TRY(ctx, hipStreamSynchronize(ex.stream));
    return C2F_OK;
}

c2f_status c2f_fbp_crown_coefficients(int32_t fuel, double out2[2]) {
    static const CrownCoef table[kNumFuels] = {C2F_CROWN_ROWS};
    if (fuel < 1 || fuel >= kNumFuels || !out2) return C2F_EINVAL;
    out2[0] = table[fuel].cbh;
    out2[1] = table[fuel].cfl;
    return C2F_OK;
}

c2f_status c2f_set_landscape_fbp(c2f_ctx* ctx, int32_t landscape_id, float fmc_pct, float pdf_pct) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, C2F_EDEVICE, "hipSetDevice failed");
    if (!(fmc_pct > 0.f && fmc_pct <= 300.f)) return fail(ctx, C2F_EINVAL, "fmc_pct must be in (0, 300]");
    if (!(pdf_pct >= 0.f && pdf_pct <= 100.f)) return fail(ctx, C2F_EINVAL, "pdf_pct must be in [0, 100]");
    std::lock_guard<std::mutex> lk2(ctx->objmu);
    auto it = ctx->lands.find(landscape_id);
    if (it == ctx->lands.end()) return fail(ctx, C2F_ESTATE, "unknown landscape id %d", landscape_id);
    Landscape& L = it->second;
    if (L.inflight > 0) return fail(ctx, C2F_EBUSY, "landscape %d is used by submitted requests", landscape_id);
    HIP_TRY(ctx, launch_fbp_consts(L.land, fmc_pct, pdf_pct, ctx->main.stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->main.stream));
    L.fmc = fmc_pct;
    L.pdf = pdf_pct;
    return C2F_OK;
}

c2f_status c2f_fbp_coefficients(int32_t fuel, double out5[5]) {
    static const FuelCoef table[kNumFuels] = {C2F_FUEL_ROWS};
    if (fuel < 1 || fuel >= kNumFuels || !out5) return C2F_EINVAL;
    out5[0] = table[fuel].a;
    out5[1] = table[fuel].b;
    out5[2] = table[fuel].c;
    out5[3] = table[fuel].q;
    out5[4] = table[fuel].bui0;
    return C2F_OK;
}

c2f_status c2f_set_tuning(c2f_ctx* ctx, int32_t block_threads, int64_t list_capacity) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    if (block_threads != 0 && block_threads != 64 && block_threads != 128 && block_threads != 256 &&
        block_threads != 512 && block_threads != 768 && block_threads != 1024)
        return fail(ctx, C2F_EINVAL, "block_threads must be 0 or one of 64,128,256,512,768,1024");
    if (list_capacity < 0 || list_capacity > ((int64_t)1 << 30))
        return fail(ctx, C2F_EINVAL, "list_capacity out of range");
    std::lock_guard<std::mutex> lk(ctx->tunemu);
    ctx->block_override = block_threads;
    ctx->cap_override = list_capacity;
    return C2F_OK;
}

c2f_status c2f_set_rep_order(c2f_ctx* ctx, int32_t mode) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    if (mode < 0 || mode > 1) return fail(ctx, C2F_EINVAL, "mode must be 0 or 1");
    std::lock_guard<std::mutex> lk(ctx->tunemu);
    ctx->rep_order = mode;
    return C2F_OK;
}

c2f_status c2f_autotune(c2f_ctx* ctx, const c2f_sim_params* rep) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Landscape* L;
    Weather* W;
    c2f_status st = check_params(ctx, rep, &L, &W);
    if (st != C2F_OK) return st;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    Exec& ex = ctx->main;
    const int64_t n = L->ncells();
    uint32_t* counts = nullptr;
    st = dev_alloc(ctx, (void**)&counts, (size_t)n * 4);
    if (st != C2F_OK) return st;
    c2f_outputs o;
    memset(&o, 0, sizeof o);
    o.burn_count = counts;
    o.on_device = 1;
    int32_t saved_block;
    int64_t saved_cap;
    auto set_over = [&](int32_t b, int64_t c) {
        std::lock_guard<std::mutex> lk2(ctx->tunemu);
        ctx->block_override = b;
        ctx->cap_override = c;
    };
    {
        std::lock_guard<std::mutex> lk2(ctx->tunemu);
        saved_block = ctx->block_override;
        saved_cap = ctx->cap_override;
    }
    // first run at the default settings finds the list high-water mark
    set_over(0, 0);
    st = simulate_impl(ctx, 1, rep, &o, false);
    int64_t cap = ex.last.list_capacity;
    const int64_t hw = (int64_t)ex.rc_host->c[kCntMaxList];
    if (st == C2F_OK && hw > 0) cap = std::max<int64_t>(1024, std::min<int64_t>(cap, 4 * hw));
    int32_t best_block = 256;
    double best_ms = 1e30;
    const int blocks[6] = {64, 128, 256, 512, 768, 1024};
    for (int b = 0; b < 6 && st == C2F_OK; ++b) {
        set_over(blocks[b], cap);
        double ms_sum = 0;
        for (int t = 0; t < 2 && st == C2F_OK; ++t) {
            st = simulate_impl(ctx, 1, rep, &o, false);
            ms_sum += ex.last.kernel_ms;
            if (ex.last.relaunches) cap = ex.last.list_capacity;
        }
        if (st == C2F_OK && ms_sum < best_ms) {
            best_ms = ms_sum;
            best_block = blocks[b];
        }
    }
    set_over(saved_block, saved_cap);
    dev_free(ctx, counts, (size_t)n * 4);
    if (st != C2F_OK) return st;
    std::lock_guard<std::mutex> lk2(ctx->tunemu);
    ctx->tune[TuneKey{n, rep->reps, rep->precision}] = TuneVal{best_block, cap};
    return C2F_OK;
}

c2f_status c2f_save_tuning(c2f_ctx* ctx, const char* path) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    if (!path || !*path) return fail(ctx, C2F_EINVAL, "no path");
    std::map<TuneKey, TuneVal> tune;
    {
        std::lock_guard<std::mutex> lk(ctx->tunemu);
        tune = ctx->tune;
    }
    // written next to the target and renamed over it, so that a reader
    // never sees a half-written file
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(ctx, C2F_EIO, "cannot write %s", tmp.c_str());
    bool ok = std::fprintf(f, "c2f-tuning 1 %s %d\n", ctx->arch.c_str(), ctx->n_cu) > 0;
    for (const auto& kv : tune)
        ok = ok && std::fprintf(f, "%lld %d %d %d %lld\n", (long long)kv.first.cells, kv.first.reps,
                                kv.first.precision, kv.second.block, (long long)kv.second.list_cap) > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(ctx, C2F_EIO, "cannot write %s", path);
    }
    return C2F_OK;
}

c2f_status c2f_load_tuning(c2f_ctx* ctx, const char* path) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    if (!path || !*path) return fail(ctx, C2F_EINVAL, "no path");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(ctx, C2F_EIO, "cannot read %s", path);
    std::map<TuneKey, TuneVal> got;
    char line[512];
    int lineno = 0;
    c2f_status st = C2F_OK;
    while (st == C2F_OK && std::fgets(line, sizeof line, f)) {
        ++lineno;
        if (!std::strchr(line, '\n') && !std::feof(f)) {
            st = fail(ctx, C2F_EINVAL, "%s:%d: line too long", path, lineno);
            break;
        }
        int used = 0;
        if (lineno == 1) {
            char arch[64];
            int version = 0, n_cu = 0;
            if (std::sscanf(line, "c2f-tuning %d %63s %d %n", &version, arch, &n_cu, &used) != 3 ||
                line[used] != '\0' || version != 1)
                st = fail(ctx, C2F_EINVAL, "%s: not a tuning file of version 1", path);
            else if (ctx->arch != arch || n_cu != ctx->n_cu)
                st = fail(ctx, C2F_EINVAL, "%s: tuned on %s with %d compute units, this device is %s with %d", path,
                          arch, n_cu, ctx->arch.c_str(), ctx->n_cu);
            continue;
        }
        long long cells = 0, cap = 0;
        int reps = 0, precision = 0, block = 0;
        if (std::sscanf(line, "%lld %d %d %d %lld %n", &cells, &reps, &precision, &block, &cap, &used) != 5 ||
            line[used] != '\0') {
            st = fail(ctx, C2F_EINVAL, "%s:%d: expected <cells> <reps> <precision> <block> <capacity>", path, lineno);
            break;
        }
        const bool block_ok = block == 64 || block == 128 || block == 256 || block == 512 || block == 768 ||
                              block == 1024;
        if (cells < 1 || reps < 1 || precision < 0 || precision > 1 || !block_ok || cap < 1 || cap > (1LL << 30)) {
            st = fail(ctx, C2F_EINVAL, "%s:%d: value out of range", path, lineno);
            break;
        }
        got[TuneKey{(int64_t)cells, reps, precision}] = TuneVal{block, (int64_t)cap};
    }
    const bool read_error = std::ferror(f) != 0;
    std::fclose(f);
    if (st != C2F_OK) return st;
    if (read_error) return fail(ctx, C2F_EIO, "cannot read %s", path);
    if (lineno == 0) return fail(ctx, C2F_EINVAL, "%s: empty file", path);
    std::lock_guard<std::mutex> lk(ctx->tunemu);
    for (const auto& kv : got) ctx->tune[kv.first] = kv.second;
    return C2F_OK;
}

c2f_status c2f_get_stats(const c2f_ctx* ctx, c2f_run_stats* out) {
    if (!ctx || !out) return C2F_EINVAL;
    *out = ctx->main.last;
    return C2F_OK;
}

// ------------------------------------------------------------- serving

c2f_status c2f_set_serving(c2f_ctx* ctx, int32_t lanes, int32_t max_batch_reps, int32_t max_batch_grid,
                           uint64_t admit_bytes) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    if (ctx->budget && admit_bytes > ctx->budget)
        return fail(ctx, C2F_EINVAL, "admit_bytes exceeds the context's budget");
    if (lanes < 1 || lanes > 16) return fail(ctx, C2F_EINVAL, "lanes must be in 1..16");
    if (max_batch_reps < 1) return fail(ctx, C2F_EINVAL, "max_batch_reps must be >= 1");
    if (max_batch_grid < 0) return fail(ctx, C2F_EINVAL, "max_batch_grid must be >= 0");
    std::lock_guard<std::mutex> lk(ctx->smu);
    if (!ctx->lanes.empty()) return fail(ctx, C2F_ESTATE, "serving already started");
    ctx->n_lanes = lanes;
    ctx->max_batch_reps = max_batch_reps;
    ctx->max_batch_grid = max_batch_grid;
    if (admit_bytes) ctx->admit_limit = admit_bytes;
    return C2F_OK;
}

c2f_status c2f_get_memory(c2f_ctx* ctx, uint64_t* bytes_held, uint64_t* admit_limit) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    if (!bytes_held || !admit_limit) return fail(ctx, C2F_EINVAL, "outputs must be non-NULL");
    *bytes_held = bytes_in_use(ctx);
    std::lock_guard<std::mutex> lk(ctx->smu);
    *admit_limit = ctx->admit_limit;
    return C2F_OK;
}

c2f_status c2f_submit(c2f_ctx* ctx, const c2f_sim_params* params, const c2f_outputs* out, uint64_t* ticket) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    if (!params || !out || !ticket) return fail(ctx, C2F_EINVAL, "params, out and ticket must be non-NULL");
    auto t = std::make_shared<Ticket>();
    t->params = *params;
    t->out = *out;
    if (params->ignition_mode == 4 && params->ignition_list && params->n_ignitions > 0 &&
        params->n_ignitions <= kMaxIgnitions) {
        t->ign_list.assign(params->ignition_list, params->ignition_list + 2 * params->n_ignitions);
        t->params.ignition_list = t->ign_list.data();
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        c2f_status st = check_params(ctx, params, &t->L, &t->W);
        if (st != C2F_OK) return st;
        std::lock_guard<std::mutex> lk2(ctx->objmu);
        ++t->L->inflight;
        ++t->W->inflight;
    }
    auto release = [&]() {
        std::lock_guard<std::mutex> lk(ctx->objmu);
        --t->L->inflight;
        --t->W->inflight;
    };
    {
        std::lock_guard<std::mutex> lk(ctx->smu);
        if ((int32_t)ctx->queue.size() >= ctx->max_queue) {
            release();
            return fail(ctx, C2F_EBUSY, "serving queue full (%d waiting)", ctx->max_queue);
        }
        if (ctx->stopping) {
            release();
            return fail(ctx, C2F_ESTATE, "context is being destroyed");
        }
        if (hipSetDevice(ctx->device) != hipSuccess) {
            release();
            return fail(ctx, C2F_EDEVICE, "hipSetDevice failed");
        }
        c2f_status st = start_lanes(ctx);
        if (st != C2F_OK) {
            release();
            return st;
        }
        t->id = ctx->next_ticket++;
        t->info.submit_ms = ms_since(ctx->t0);
        ctx->tickets[t->id] = t;
        ctx->queue.push_back(t);
    }
    ctx->scv.notify_all();
    *ticket = t->id;
    return C2F_OK;
}

c2f_status c2f_poll(c2f_ctx* ctx, uint64_t ticket, int32_t* done) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    if (!done) return fail(ctx, C2F_EINVAL, "done must be non-NULL");
    std::lock_guard<std::mutex> lk(ctx->smu);
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return fail(ctx, C2F_ESTATE, "unknown ticket %llu", (unsigned long long)ticket);
    *done = it->second->done ? 1 : 0;
    return C2F_OK;
}

c2f_status c2f_wait_info(c2f_ctx* ctx, uint64_t ticket, c2f_ticket_info* info) {
    if (!ctx) return C2F_EINVAL;
    ApiScope api(ctx);
    std::unique_lock<std::mutex> lk(ctx->smu);
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return fail(ctx, C2F_ESTATE, "unknown ticket %llu", (unsigned long long)ticket);
    std::shared_ptr<Ticket> t = it->second;
    ctx->scv.wait(lk, [&] { return t->done; });
    ctx->tickets.erase(ticket);
    if (info) *info = t->info;
    if (t->status != C2F_OK) return fail(ctx, t->status, "%s", t->err.c_str());
    return C2F_OK;
}

c2f_status c2f_wait(c2f_ctx* ctx, uint64_t ticket) { return c2f_wait_info(ctx, ticket, nullptr); }

}  // extern "C"
