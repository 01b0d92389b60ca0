// Host-side launchers of the gfx950 kernels (internal to libc2f).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "types.h"

namespace c2f {

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);

// Cell records, burnable list, nearest-centre cell and landscape constants.
// tile_scratch holds tile_scratch_entries(rows*cols) int32.  Slopes come
// from elev (NULL = flat) or, when grad_from is set, from the Horn
// numerators of those records.
hipError_t launch_prepare_landscape(const uint8_t* fuel, const int16_t* elev, const CellRec* grad_from,
                                    int rows, int cols, int cell_m, float pc, float curing, float fmc,
                                    float pdf, CellRec* recs, int32_t* burnable, int32_t* tile_scratch,
                                    LandDev* land, hipStream_t s);
// Rewrite the foliar-moisture and dead-fir constants of a landscape.
hipError_t launch_fbp_consts(LandDev* land, float fmc, float pdf, hipStream_t s);

// Scar comparison in one launch: out[t] = MSE, out[T + t] = SSIM of period
// t, out[2T] = Frobenius norm of the last period's difference.  counts (3 T
// u64) and *ticket must be zero on entry and are zero again once the launch
// ends; launches sharing them must be ordered (one stream).
// 2 <= n, 1 <= T <= 65535.
hipError_t launch_scar_metrics(const int32_t* arrival, const uint8_t* reference, int64_t n, int T, int period_min,
                               unsigned long long* counts, uint32_t* ticket, double* out, hipStream_t s);

// fuel[cells[k]] = codes[k] for k < n.
hipError_t launch_fuel_edits(uint8_t* fuel, const int32_t* cells, const uint8_t* codes, int64_t n, hipStream_t s);
int64_t tile_scratch_entries(int64_t n_cells);

// Per (scenario, period) weather terms in FP64 and FP32; wx is [n_rows][4].
hipError_t launch_weather_table(const float* wx, int n_rows, double* t64, float* t32, hipStream_t s);

hipError_t launch_eval_ros(int precision, const EvalArgs& a, hipStream_t s);

// Persistent propagation over `total` work items (one per replication).
hipError_t launch_propagate(int precision, int block, int grid, const Job* jobs, int n_jobs, int total,
                            const Slots& slots, RunCounters* rc, hipStream_t s);
int propagate_blocks_per_cu(int precision, int block);

// Replication order of a launch whose work groups each run several items:
// keys[item] = predicted head-fire travel (zeroed first), order = items by
// decreasing key.  max_periods <= 65535.
hipError_t launch_order(int precision, const Job* jobs, int n_jobs, int total_items, int max_periods,
                        unsigned long long* keys, int32_t* order, hipStream_t s);

// Dense per-replication outputs of a launch whose items each kept a slot
// (slots.item_slot filled by the propagation, cleared to -1 before it);
// total <= 65535; nothing is written if the launch overflowed.
hipError_t launch_dense_outputs(const Job* jobs, int n_jobs, int total, int n_slots, int64_t max_cells,
                                const Slots& slots, const RunCounters* rc, hipStream_t s);

// Work counts of a finished request (account.hip): out[0..2] +=
// burning-cell-periods, axis reach events, ignitions, from the final arrival
// minutes [reps][rows*cols] (-1 unburned) of the request described by *job
// (device); total_cells = reps * rows * cols.
hipError_t launch_work_counts(int precision, const Job* job, int64_t total_cells, const int32_t* arrival,
                              unsigned long long* out, hipStream_t s);

// No-allocation scratch (noalloc.hip): kScratchBytes of device memory per
// device, held for the life of the process.  scratch_resolve gives the
// device address of `device`'s copy (resolved once, with that device
// current); scratch_lock serialises its users within the process.
constexpr size_t kScratchBytes = (size_t)128 << 20;
hipError_t scratch_resolve(int device, void** out);
std::mutex& scratch_lock(int device);
// *dst = j, ordered on s (the job record of a launch, without host staging).
hipError_t launch_store_job(const Job& j, Job* dst, hipStream_t s);

}  // namespace c2f
