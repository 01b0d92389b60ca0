// Plain structures shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace c2f {

// Arrival labels: 12-bit generation tag above a 20-bit minute.  A work
// slot's arrival plane is never cleared between replications; each
// replication takes a smaller tag, so every value left by an earlier one
// compares larger than any label of the current one (i.e. "not burned").
// Minute kPendingMinute marks a cell whose centre was reached while its own
// rate was below the ignition threshold (it ignites at the start of the
// first later period that passes); it compares above every real minute.
constexpr uint32_t kMinuteBits = 20;
constexpr uint32_t kMinuteMask = (1u << kMinuteBits) - 1u;
constexpr uint32_t kPendingMinute = kMinuteMask;
constexpr int32_t kMaxMinutes = (1 << kMinuteBits) - 2;   // longest run, minutes
constexpr uint32_t kTagFresh = 4095u;                       // tag of a freshly filled plane
constexpr uint32_t kPlaneFill = 0xFFFFFFFFu;

// Weather-table row: [0] f(F), [1] ISZ, [2] WS sin(WAZ), [3] WS cos(WAZ),
// [4 + f] BUI effect of fuel f, [23 + f] 1 - exp(-b_f ISZ) of pure fuel f
// (the zero-wind rate RSZ = a (1 - exp(-b ISZ))^c without its a and c),
// [42 + f] surface fuel consumption of fuel f (kg/m^2; M-1/M-2 mix the C-2
// and D-1 entries by percent conifer where it is used).  19 fuel codes.
constexpr int kRowBE = 4;
constexpr int kRowG = 23;
constexpr int kRowSFC = 42;
constexpr int kRowLen = 64;

// Static per-cell record, 32 bytes:
//   info: fuel code (bits 0-7) | mask of burnable neighbours (bits 8-15,
//         bit k = axis k: E, NE, N, NW, W, SW, S, SE)
//   grad: Horn numerators gx (int16, low half) and gn (int16, high half)
//   sfc:  SF^(1/c) for the cell's own rate curve (the C-2 curve for M-1/M-2),
//         with SF the FBP slope factor exp(3.533 (GS/100)^1.2), 10 from
//         70 % up; 1 on flat ground
//   sfd:  SF^(1/c) for the D-1 curve (M-1/M-2 cells only)
// With these, the slope-adjusted spread index of a fuel with curve
// a (1 - exp(-b ISI))^c is ISF = ln(1 - sfc (1 - exp(-b ISZ))) / -b.
struct alignas(16) CellRec {
    uint32_t info;
    uint32_t grad;
    uint32_t pad[2];
    double sfc;
    double sfd;
};

// Per-landscape values computed on the device at load time.
struct LandDev {
    int32_t n_burnable;
    int32_t centre_cell;       // burnable cell nearest (rows/2, cols/2), -1 if none
    int32_t grad_overflow;     // a Horn numerator left the int16 range
    int32_t pad0;
    unsigned long long centre_key;
    double pc_w64, cf64, cell_m64;
    float pc_w32, cf32, cell_m32, pad1;
    // percent dead fir / 100 (M-3, M-4), and the C-6 foliar moisture effect
    // relative to its average (FME / 0.778)
    double pdf_w64, fme_r64;
    float pdf_w32, fme_r32;
    // critical surface intensity for crowning per fuel (kW/m):
    // 0.001 CBH^1.5 (460 + 25.9 FMC)^1.5
    double csi64[19];
    float csi32[19];
};

// Entries of an ignition-point list carried by one request.
constexpr int kMaxIgnitions = 32;

// One simulation request as the propagation kernel sees it.
struct Job {
    const CellRec* cells;
    const int32_t* burnable;   // row-major burnable cells
    const LandDev* land;
    const void* table;         // [n_scen][n_wp][kRowLen] weather terms, double or float
    const double* table64;     // the same terms in FP64 (slope-equivalent wind)
    const float* table32;      // the same terms in FP32 (an FP64 job tries them first); may be NULL
    int32_t rows, cols, d_orth, d_diag;
    int32_t n_scen, n_wp, period_min, n_periods;
    int32_t T, reps, rep_offset, item_base;
    int32_t rounding, ign_mode, ign_cell, scen_mode;
    int32_t scen_fixed, ign_period;
    float sigma, threshold;
    uint64_t seed;
    const uint64_t* ign_cdf;   // ignition map: running weight sums per cell (mode 3)
    uint64_t ign_total;
    int32_t burn_hours;        // daily burning window (0 = always)
    float burnout;             // burn-out rate threshold, m/min (0 = off)
    float hfi_min;             // burn-out head fire intensity threshold, kW/m (0 = off)
    // ignition-point list (mode 4): (cell, period) pairs by period; each
    // cell is lit at minute period * period_min if it has not burned
    int32_t n_seeds;
    int2 seeds[kMaxIgnitions];
    uint8_t* scar;             // outputs (device); NULL = not wanted
    int32_t* arr_period;
    int32_t* arr_minute;
    uint32_t* count;
    int64_t* burned;
    int32_t* ign_out;
    int32_t* scen_out;
};

// A cell whose fire has not yet reached some neighbours by the end of a
// period: its label and the metres left on each axis (u16 pairs).
struct Cont {
    uint32_t c, label;
    uint32_t rem[4];
};

// Global part of a work slot's lists, list_cap entries each:
//   W    the period queue beyond its LDS part (2 x list_cap entries), uint2 (cell, label)
//   C[2] continuation lists, Cont
//   P[2] pending cells, uint32
constexpr int64_t kSlotListBytesPerEntry = 2 * 8 + 2 * 24 + 2 * 4;

// Replication order of a launch: a 64-bit key and a 32-bit position per item.
constexpr size_t kOrderBytesPerItem = 8 + 4;

// Work slots: one per resident work group.  Each owns an arrival plane of
// plane_cells labels, its lists and a tag.  A launch uses list_limit entries
// of each list; the buffers may hold more from an earlier, larger launch.
struct Slots {
    uint32_t* planes;
    int64_t plane_cells;
    uint8_t* lists;
    int64_t list_cap;     // entries allocated per list (layout stride)
    int64_t list_limit;   // entries a launch may use (overflow beyond it)
    uint32_t* tags;
    // When every item of a launch has a slot of its own, the per-rep dense
    // outputs (scar, arrival minute and period) are written after the
    // propagation by a grid-wide kernel: item_slot[item] = {slot, tag}.
    // NULL: each work group writes them at the end of its replication.
    int2* item_slot;
    // order[n] = the item the n-th fetch of a work group takes (longest
    // predicted replications first); NULL: item n.
    const int32_t* order;
};

enum Counter {
    kCntEntries = 0,     // queue entries read
    kCntEvals,           // per (cell, period) rate evaluations
    kCntCandidates,      // arrival candidates offered
    kCntImprovements,    // candidates that lowered a label
    kCntIgnitions,       // cells ignited
    kCntRounds,          // label-correcting rounds
    kCntConts,           // continuation entries read
    kCntMaxList,         // largest list length seen
    kNumCounters = 8
};

struct RunCounters {
    int32_t next_item;
    int32_t overflow;
    int32_t pad[2];
    unsigned long long c[kNumCounters];
};

struct EvalArgs {
    const CellRec* cells;
    const LandDev* land;
    const void* table;
    const double* table64;
    const float* table32;
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
    double* cfb;
    double* hfi;
};

}  // namespace c2f
