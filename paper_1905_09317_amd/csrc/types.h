// Plain structures shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace c2f {

// Arrival labels: 12-bit generation tag above a 20-bit minute.  A work
// slot's arrival plane is never cleared between replications; each
// replication takes a smaller tag, so every value left by an earlier one
// compares larger than any label of the current one (i.e. "not burned").
constexpr uint32_t kMinuteBits = 20;
constexpr uint32_t kMinuteMask = (1u << kMinuteBits) - 1u;
constexpr int32_t kMaxMinutes = (1 << kMinuteBits) - 2;   // longest run, minutes
constexpr uint32_t kTagFresh = 4095u;                       // tag of a freshly filled plane
constexpr uint32_t kPlaneFill = 0xFFFFFFFFu;

// Weather-table row: [0] f(F), [1] ISZ, [2] WS sin(WAZ), [3] WS cos(WAZ),
// [4 + f] BUI effect of fuel f, [20 + f] zero-wind rate of pure fuel f.
constexpr int kRowLen = 36;
constexpr int kRowBE = 4;
constexpr int kRowRSZ = 20;

// Per-landscape values computed on the device at load time.
struct LandDev {
    int32_t n_burnable;
    int32_t centre_cell;       // burnable cell nearest (rows/2, cols/2), -1 if none
    int32_t grad_overflow;     // a Horn numerator left the int16 range
    int32_t pad0;
    unsigned long long centre_key;
    double pc_w64, cf64, cell_m64;
    float pc_w32, cf32, cell_m32, pad1;
};

// One simulation request as the propagation kernel sees it.
struct Job {
    const uint8_t* fuel;
    const uint32_t* grad;      // (gx int16) | (gn int16) << 16
    const int32_t* burnable;   // row-major burnable cells
    const LandDev* land;
    const void* table;         // [n_scen][n_wp][kRowLen] weather terms, double or float
    const double* table64;     // the same terms in FP64 (slope-equivalent wind)
    int32_t rows, cols, d_orth, d_diag;
    int32_t n_scen, n_wp, period_min, n_periods;
    int32_t T, reps, rep_offset, item_base;
    int32_t rounding, ign_mode, ign_cell, scen_mode;
    int32_t scen_fixed, pad0;
    float sigma, threshold;
    uint64_t seed;
    uint8_t* scar;             // outputs (device); NULL = not wanted
    int32_t* arr_period;
    int32_t* arr_minute;
    uint32_t* count;
    int64_t* burned;
    int32_t* ign_out;
    int32_t* scen_out;
};

// Work slots: one per resident work group.  Each owns an arrival plane of
// plane_cells labels, four work lists of list_cap entries and a tag.
struct Slots {
    uint32_t* planes;
    int64_t plane_cells;
    uint2* lists;
    int64_t list_cap;
    uint32_t* tags;
};

enum Counter {
    kCntEntries = 0,
    kCntEvals,
    kCntCandidates,
    kCntImprovements,
    kCntIgnitions,
    kCntMaxList,
    kNumCounters = 8
};

struct RunCounters {
    int32_t next_item;
    int32_t overflow;
    int32_t pad[2];
    unsigned long long c[kNumCounters];
};

struct EvalArgs {
    const uint8_t* fuel;
    const uint32_t* grad;
    const LandDev* land;
    const void* table;
    const double* table64;
    int32_t n_cells, scenario, period, n_wp;
    uint32_t rep;
    int32_t rounding;
    float sigma;
    uint64_t seed;
    double* hros;
    double* bros;
    double* fros;
    double* lb;
    double* raz;
    double* x8;
    int32_t* q8;
};

}  // namespace c2f
