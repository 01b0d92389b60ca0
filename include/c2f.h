/*
 * c2f.h -- C ABI of libc2f.so, an MI355X (gfx950) implementation of the
 * Cell2Fire fire-growth hot path (Pais, Carrasco, Martell, Weintraub,
 * Woodruff, "Cell2Fire: A Cell Based Forest Fire Growth Model").
 *
 * What the library computes
 *   A landscape is a rectangular grid of square cells, each with a fuel type
 *   and an elevation (Section 3.1; inputs of Section 3.5).  For every burning
 *   cell and weather period it evaluates the FBP System head, back and flank
 *   rates and length-to-breadth ratio (Sections 2.3 and 3.7, assumption A2),
 *   fits the ellipse of eqs. (2)-(4), and spreads fire along the 8
 *   centre-to-centre axes at the rate of eq. (1).  A neighbour whose centre
 *   is reached receives a message and ignites if its own rate passes the
 *   threshold (Section 3.1; Algorithm 1 Step 2).  The clock advances in
 *   whole minutes; weather changes every period.  Many stochastic
 *   replications (ROS noise, weather scenario, ignition cell; Section 3.1,
 *   sources of uncertainty (1)-(3)) are run and folded into burn-count maps
 *   (Section 3.6 (i)).
 *
 * Conventions shared by all entry points
 *   - Grids are row-major, row 0 is the northern edge, cell index
 *     i = row * cols + col.  Axis order everywhere: E, NE, N, NW, W, SW, S,
 *     SE (0 deg = East, counter-clockwise, Section 3.4 step i).
 *   - Fuel codes: 0 non-fuel, 1-7 C-1..C-7, 8 D-1, 9 M-1, 10 M-2,
 *     11-13 S-1..S-3, 14 O-1a, 15 O-1b, 16 D-2, 17 M-3, 18 M-4 (Table FBPT
 *     gives the dictionary idea; Section 2.3 lists the FBP fuel types).
 *   - Every function returns a c2f_status; nothing is thrown or aborted
 *     across the ABI.  On failure, outputs are not written and
 *     c2f_last_error() describes the cause.
 *   - Host pointers passed in are only read during the call; the library
 *     copies what it keeps.  All device memory is owned by the context and
 *     released by c2f_destroy().
 *   - Entry points may be called from several threads: synchronous calls
 *     on one context are serialised; served requests run on their own lanes
 *     beside them.
 *   - Results depend only on (landscape, weather, params including seed):
 *     never on block size, batch composition or co-resident work.
 */
#ifndef C2F_H
#define C2F_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    C2F_OK = 0,
    C2F_EINVAL = -1,    /* bad argument, shape or value */
    C2F_ENOMEM = -2,    /* device allocation failed or HBM budget exceeded */
    C2F_EDEVICE = -3,   /* HIP runtime error or no suitable device */
    C2F_ECAPACITY = -4, /* work lists overflowed even at the largest capacity */
    C2F_ESTATE = -5,    /* unknown landscape/weather id or ticket, or wrong call order */
    C2F_EBUSY = -6,     /* serving queue is full */
    C2F_EIO = -7        /* a file could not be opened, read or written */
} c2f_status;

typedef struct c2f_ctx c2f_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the
 * device memory the context may hold (0 = no cap beyond the device).
 * Loads the code object and allocates nothing else yet. */
c2f_status c2f_create(int32_t device, uint64_t hbm_budget_bytes, c2f_ctx** out);

/* Release every device allocation and the context.  NULL is allowed. */
void c2f_destroy(c2f_ctx* ctx);

/* Text of the last error on this context (empty if none).  Valid until the
 * next call on the context. */
const char* c2f_last_error(const c2f_ctx* ctx);

/* Order all later synchronous work on `hip_stream` (a hipStream_t, e.g.
 * torch's current stream); NULL selects the context's own stream, a
 * blocking stream that is ordered with the legacy null stream.  Default
 * priority only. */
c2f_status c2f_set_stream(c2f_ctx* ctx, void* hip_stream);

/* Upload a landscape (Section 3.5 (i)): fuel codes [rows*cols] (host) and
 * elevations in metres [rows*cols] (host; NULL = flat ground).  cell_m is
 * the cell width in metres (1..20000).  pc_pct is the percent conifer of
 * M-1/M-2 stands (0..100), curing_pct the grass curing of O-1 (0 < c <= 100).
 * Slope (percent) and upslope azimuth are derived on the device from Horn's
 * 3x3 gradient with replicated edges; EINVAL if a gradient numerator
 * exceeds the int16 range (a rise of more than ~4 km across one cell).
 * Writes a new id to *landscape_id. */
c2f_status c2f_load_landscape(c2f_ctx* ctx, int32_t rows, int32_t cols, int32_t cell_m,
                              const uint8_t* fuel, const int16_t* elev_m, float pc_pct,
                              float curing_pct, int32_t* landscape_id);
c2f_status c2f_unload_landscape(c2f_ctx* ctx, int32_t landscape_id);

/* FBP inputs of a loaded landscape besides percent conifer and curing
 * (Section 2.3: the FBP System's fuel moisture and stand descriptors):
 * foliar moisture content fmc_pct (0 < FMC <= 300; default 97, where the C-6
 * foliar moisture effect equals its average) for C-6 crown fire and the
 * crown fraction burned of every crowning fuel, and percent dead fir
 * pdf_pct (0..100, default 50) of M-3/M-4 stands.  Derived landscapes take
 * their base's values.  EBUSY while the landscape is used by submitted
 * requests. */
c2f_status c2f_set_landscape_fbp(c2f_ctx* ctx, int32_t landscape_id, float fmc_pct, float pdf_pct);

/* A treatment variant of a loaded landscape (Section 1: harvested or
 * non-fuel cells as fuel-management plans): a new landscape with the base's
 * grid, elevation (its slopes are taken from the base's cell records), cell
 * width, percent conifer and curing, and fuel[cells[k]] = fuels[k] for the
 * n_edits edits (fuel 0 = harvested / non-fuel; later edits of a cell win).
 * Cell records, burnable list and centre cell are rebuilt on the device.
 * The base's ignition map is not carried over.  Plans of one base share a
 * launch through c2f_simulate_batch; each plan's burn_count / reps is its
 * burn-probability map. */
c2f_status c2f_derive_landscape(c2f_ctx* ctx, int32_t base_id, int64_t n_edits, const int32_t* cells,
                                const uint8_t* fuels, int32_t* landscape_id);

/* Scar comparison (Section 4, comparison methodology).  For t = 1..n_periods
 * the simulated scar Y^t = {cells with arrival_minute in [0, t period_min]}
 * (one replication's arrival_minute output, -1 = unburned) is compared with
 * the reference 0-1 scar X^t = reference[t-1][.] ([n_periods][n_cells],
 * nonzero = burned): mse[t-1] = mean (X - Y)^2; ssim[t-1] = the structural
 * similarity of Wang et al. (2004) over the whole grid, ((2 mu_x mu_y + C1)
 * (2 sigma_xy + C2)) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)),
 * C1 = 1e-4, C2 = 9e-4, (co)variances normalised by N - 1; *delta_norm =
 * the Frobenius norm of X - Y at the last period.  Inputs are device
 * pointers when on_device, else host (copied); outputs are host arrays
 * (any may be NULL).  Synchronous on the context's stream.
 * 2 <= n_cells < 2^31, 1 <= n_periods <= 65535. */
c2f_status c2f_compare_scars(c2f_ctx* ctx, int64_t n_cells, int32_t n_periods, int32_t period_min,
                             const int32_t* arrival_minute, const uint8_t* reference, int32_t on_device,
                             double* mse, double* ssim, double* delta_norm);

/* The same comparison ordered on the context's stream without waiting, for
 * callers that keep the results in device memory: arrival_minute,
 * reference and results are device pointers; results receives [2 n_periods
 * + 1] doubles (mse, then ssim, then delta_norm) once the stream reaches
 * the work.  The context keeps its count buffer between calls, so calls on
 * one stream follow each other safely; calls of one context on different
 * streams (c2f_set_stream between them) must not overlap.  The argument
 * checks of c2f_compare_scars apply. */
c2f_status c2f_compare_scars_async(c2f_ctx* ctx, int64_t n_cells, int32_t n_periods, int32_t period_min,
                                   const int32_t* arrival_minute, const uint8_t* reference, double* results);

/* Spatial ignition probability of a landscape (Section 3.1, uncertainty
 * (1)): weights[rows*cols] (host, row-major, copied) give cell i the
 * probability weights[i] / sum(weights) under ignition_mode 3.  The draw is
 * integer: with x the 32-bit Philox word of tag 3 and W the sum, the target
 * floor(x W / 2^32) selects the first cell whose running sum exceeds it.  A
 * cell without fuel may be drawn and then burns nothing; an all-zero map
 * ignites nothing.  weights == NULL removes the map.  EBUSY while the
 * landscape is used by submitted requests. */
c2f_status c2f_set_ignition_map(c2f_ctx* ctx, int32_t landscape_id, const uint32_t* weights);

/* One weather record (Table WeatherT columns used by the FBP System):
 * FFMC (0..101), BUI (>= 0), wind speed km/h (>= 0) and the azimuth the
 * wind blows FROM, degrees clockwise from north. */
typedef struct {
    float ffmc, bui, ws_kmh, wd_deg_from;
} c2f_weather_row;

/* Upload weather scenarios (Section 3.5 (iv)): rows [n_scen][n_periods]
 * (host), one record per period of period_min minutes.  Writes an id. */
c2f_status c2f_set_weather(c2f_ctx* ctx, int32_t n_scen, int32_t n_periods, int32_t period_min,
                           const c2f_weather_row* rows, int32_t* weather_id);
c2f_status c2f_unset_weather(c2f_ctx* ctx, int32_t weather_id);

/* Parameters of one Monte-Carlo simulation request.
 *   reps           replications (>= 1); rep index r uses the global index
 *                  rep_offset + r in every random draw, so a run split into
 *                  rep ranges reproduces the unsplit run exactly.
 *   n_periods      fire periods to simulate (<= the weather's periods);
 *                  the fire runs for n_periods * period_min minutes.
 *   seed           Philox4x32-10 key (low word, high word).
 *   ros_sigma      lognormal ROS noise: every rate of a cell in a period is
 *                  multiplied by exp(sigma Z - sigma^2/2) (0 = off).
 *   ros_threshold  a reached cell ignites only if its head rate exceeds this
 *                  (m/min; Section 3.1); otherwise it stays reached and
 *                  ignites at the start of the first later period that passes.
 *   rounding       axis rates are integer m/min: 0 = floor(x + 1/2),
 *                  1 = floor(x + u) with u uniform from Philox.
 *   precision      0 = FP64 results: the integer rates (and the intensity
 *                  burn-out test) are those of an FP64 evaluation.  Each
 *                  cell is evaluated in FP32 first; where x + u lies
 *                  within 3e-5 max(1, x) of an integer, the intensity
 *                  within 2e-4 of its threshold, or the wind speed within
 *                  1e-3 km/h of a switch of the model's form (40 km/h,
 *                  and 1 km/h for grass), the FP64 evaluation decides.
 *                  1 = FP32 rates throughout.
 *   ignition_mode  0 = ignition_cell, 1 = uniform over burnable cells,
 *                  2 = the burnable cell nearest (rows/2, cols/2),
 *                  3 = drawn from the landscape's ignition map
 *                  (c2f_set_ignition_map; Section 3.1, uncertainty (1)),
 *                  4 = the ignition-point list below.
 *   scenario_mode  0 = scenario, 1 = uniform over the weather's scenarios.
 *   ignition_period  the fire is lit at the start of this period
 *                  (0 <= ignition_period < n_periods): its cell takes minute
 *                  ignition_period * period_min, and minute m belongs to
 *                  period (m - 1) / period_min, so a later ignition reads as
 *                  the period before it in arrival_period.
 *   burn_hours     maximum burning hours per day (assumption A5): 0 or 24
 *                  = no limit; 1..23 = fire spreads and cells ignite only
 *                  in the first burn_hours hours of every day counted from
 *                  the start of the run (progress pauses outside them).
 *                  Needs a period length that divides 60 minutes.
 *   burnout_ros    burn-out threshold delta (m/min; assumption A5 (i); 0 =
 *                  off): when a burning cell's rates are evaluated for a
 *                  period and its integer axis rates toward every in-grid
 *                  burnable neighbour are below delta, it spreads no further,
 *                  in that period or later.
 *   n_ignitions, ignition_list  the ignition-point input of Section 3.2
 *                  (iii) for ignition_mode 4: n_ignitions (1..32) pairs
 *                  (cell, period) (host, copied; 0 <= period < n_periods, any
 *                  order).  Every replication lights each listed cell at
 *                  minute period * period_min, as a single ignition at that
 *                  period would be, if the cell has fuel and has not burned
 *                  yet (a reached cell waiting on the threshold included),
 *                  inside or outside the burning window; the run goes on
 *                  while entries remain.  ignition_period is unused, and the
 *                  replication's reported ignition is the cell of the
 *                  earliest entry (the first listed among entries of one
 *                  period).  Other modes need n_ignitions = 0.
 *   hfi_min        head fire intensity threshold (kW/m; assumption A5 (iv);
 *                  0 = off): when a burning cell's rates are evaluated for a
 *                  period and its head fire intensity 300 TFC ROS (total
 *                  fuel consumption from the FBP System, ROS the head rate
 *                  with the noise multiplier) is below it, it spreads no
 *                  further, in that period or later.  In precision 1 the
 *                  intensity is compared in FP32. */
typedef struct {
    int32_t landscape_id, weather_id, reps, n_periods;
    uint64_t seed;
    float ros_sigma, ros_threshold;
    int32_t rounding, precision;
    int32_t ignition_mode, ignition_cell;
    int32_t scenario_mode, scenario;
    int32_t rep_offset;
    int32_t ignition_period, burn_hours;
    float burnout_ros;
    int32_t n_ignitions;
    const int32_t* ignition_list;
    float hfi_min;
} c2f_sim_params;

/* Outputs of a simulation (Section 3.6 (i) burn grids and their counts).
 * Any pointer may be NULL (not wanted).  With on_device = 0 they are host
 * pointers; with 1 they are device pointers (e.g. torch tensors'
 * data_ptr()) written in order on the context's stream.
 *   scar           uint8  [reps][rows*cols]  1 = ignited within the run
 *   arrival_period int32  [reps][rows*cols]  -1 unburned, 0 ignition cell,
 *                                            else (minute - 1) / period_min
 *   arrival_minute int32  [reps][rows*cols]  -1 unburned, else minute
 *   burn_count     uint32 [rows*cols]        number of reps that burned it
 *   burned_cells   int64  [reps]             cells burned per rep
 *   ignition_cell  int32  [reps]             -1 if no burnable cell
 *   scenario       int32  [reps]                                           */
typedef struct {
    uint8_t* scar;
    int32_t* arrival_period;
    int32_t* arrival_minute;
    uint32_t* burn_count;
    int64_t* burned_cells;
    int32_t* ignition_cell;
    int32_t* scenario;
    int32_t on_device;
} c2f_outputs;

/* Run one simulation request to completion (synchronous). */
c2f_status c2f_simulate(c2f_ctx* ctx, const c2f_sim_params* params, const c2f_outputs* out);

/* Run several requests, possibly on different landscapes and weather, in
 * one fused launch (synchronous).  params[n_jobs], out[n_jobs]. */
c2f_status c2f_simulate_batch(c2f_ctx* ctx, int32_t n_jobs, const c2f_sim_params* params,
                              const c2f_outputs* out);

/* c2f_simulate for callers that cannot allocate device memory (code that
 * runs while a HIP graph is being captured, tight serving loops, hosts that
 * forbid allocation after start-up).  It calls no hipMalloc, hipFree or
 * other allocating routine: the launch's counters, job record, generation
 * tags, arrival planes and work lists live in a fixed device scratch array
 * of 128 MiB that the library's code object holds on every device it runs
 * on until the process ends (its address is resolved once per device by
 * c2f_create).  Outputs must be device pointers (out->on_device = 1), written
 * in order on the context's stream; the call returns once they are complete.
 * Results equal c2f_simulate's for the same request.  EINVAL if one work
 * slot (an arrival plane of 4 B per cell plus its work lists) does not fit
 * the scratch; the request then needs c2f_simulate.  Fewer resident work
 * groups than c2f_simulate may run when the scratch holds fewer slots, and
 * work lists start small and grow on overflow (ECAPACITY past the largest
 * size that fits), which changes no result.  The scratch keeps whatever the
 * last call left in it; each call first resets the state it reads.  Calls
 * on one device share the scratch: the library serialises them within a
 * process, and calls that overlapped on one device would race. */
c2f_status c2f_simulate_noalloc(c2f_ctx* ctx, const c2f_sim_params* params, const c2f_outputs* out);

/* Work counts of a finished request, for measuring the algorithmic bytes of
 * the sending stage (Section 3.8, App. A; Algorithm 1 Step 2).  From the
 * request's final arrival minutes (arrival_minute output of c2f_simulate
 * with the same params: device pointer, int32 [reps][rows*cols], -1 =
 * unburned) it writes counts[0] = burning-cell-periods, the (replication,
 * cell, period) triples whose rates the cell takes while some axis still
 * leads to a neighbour that has not ignited; counts[1] = axis reach events,
 * progress along an axis reaching the neighbour's centre before it ignites;
 * counts[2] = ignitions (burned cells).  These are the minute-stepping
 * loop's own units, independent of how the simulation ordered its work.
 * Synchronous on the context's stream; counts is a host array of 3. */
c2f_status c2f_count_work(c2f_ctx* ctx, const c2f_sim_params* params, const int32_t* arrival_minute,
                          int64_t* counts);

/* Parity/debug: the per-cell FBP field of one (scenario, period, rep) on the
 * landscape, exactly as the simulation computes it.  Host outputs, any may
 * be NULL, each [rows*cols] (q8 and x8: [rows*cols][8]):
 * hros/bros/fros m/min including the rep's noise multiplier, lb, raz_deg
 * (spread azimuth, clockwise from north), x8 the unquantised axis rates
 * (eq. (1) times the multiplier), q8 the integer axis rates, cfb the crown
 * fraction burned and hfi the head fire intensity (kW/m, with the
 * multiplier on the rate).  Non-fuel cells give zeros. */
c2f_status c2f_eval_ros(c2f_ctx* ctx, int32_t landscape_id, int32_t weather_id, int32_t scenario,
                        int32_t period, int32_t rep, uint64_t seed, float sigma, int32_t rounding,
                        int32_t precision, double* hros, double* bros, double* fros, double* lb,
                        double* raz_deg, double* x8, int32_t* q8, double* cfb, double* hfi);

/* FBP coefficients (a, b, c, q, BUI0) of fuel code 1..18 as the device uses
 * them (M-1/M-2 report zeros for a, b, c; M-3/M-4 their dead-fir curves).
 * Host-only, needs no device. */
c2f_status c2f_fbp_coefficients(int32_t fuel, double out5[5]);

/* Crown base height (m) and crown fuel load (kg/m^2) of fuel code 1..18
 * (zeros for fuels that do not crown).  Host-only. */
c2f_status c2f_fbp_crown_coefficients(int32_t fuel, double out2[2]);

/* Tuning.  block_threads: threads per work group of the propagation kernel
 * (one of 64, 128, 256, 512, 768, 1024; 0 = automatic).  list_capacity: least number
 * of entries per per-replication work list (0 = automatic).  A too small
 * capacity is detected and the run repeated with a larger one, so results
 * never change. */
c2f_status c2f_set_tuning(c2f_ctx* ctx, int32_t block_threads, int64_t list_capacity);

/* Replication order.  When a launch has more replications than resident
 * work groups, each group runs several one after another, and a long
 * replication taken last keeps its group busy after the others finish.
 * mode 1 (default): before the launch, a small kernel predicts each
 * replication's length from the head rate at its ignition cell over the
 * run (Sections 3.1 and 3.4) and groups take the longest first; mode 0:
 * index order.  Only the schedule changes: every replication keeps its
 * index, random streams and output row, so results are identical. */
c2f_status c2f_set_rep_order(c2f_ctx* ctx, int32_t mode);

/* Pick block size and list capacity for requests like `representative` by
 * timing candidates on the device; the choice is kept for requests of the
 * same grid size and replication count. */
c2f_status c2f_autotune(c2f_ctx* ctx, const c2f_sim_params* representative);

/* Tuning cache on disk, so that a choice made by c2f_autotune (or a list
 * capacity raised after an overflow) carries over to later contexts and
 * processes.  c2f_save_tuning writes every entry the context holds to the
 * text file `path` (replaced whole); c2f_load_tuning reads such a file and
 * adds its entries to the context (an entry for the same grid size,
 * replication count and precision replaces the context's).  The file names
 * the device it was tuned on (architecture and compute-unit count) and one
 * entry per line:
 *   c2f-tuning 1 <arch> <compute units>
 *   <cells> <replications> <precision> <block threads> <list capacity>
 * Loading a file tuned on another kind of device, or a malformed file,
 * fails with C2F_EINVAL and changes nothing; a missing file is C2F_EIO.
 * Block sizes must be one of 64, 128, 256, 512, 768, 1024 and list
 * capacities 1 .. 2^30. */
c2f_status c2f_save_tuning(c2f_ctx* ctx, const char* path);
c2f_status c2f_load_tuning(c2f_ctx* ctx, const char* path);

/* Counters of the most recent simulate/simulate_batch call. */
typedef struct {
    int64_t ignitions;       /* cells ignited, summed over reps */
    int64_t entries;         /* work-list entries processed (incl. stale) */
    int64_t rate_evals;      /* per (cell, period) rate evaluations */
    int64_t candidates;      /* arrival candidates offered to neighbours */
    int64_t improvements;    /* candidates that lowered an arrival */
    int64_t relaunches;      /* repeats after a work-list overflow */
    int64_t rounds;          /* label-correcting rounds, summed over reps */
    int64_t continuations;   /* period-boundary continuations read */
    double kernel_ms;        /* propagation kernel time (HIP events) */
    int32_t block_threads, grid_blocks;
    int64_t list_capacity;
    int32_t rep_order;       /* 1 if groups took replications longest-predicted first */
} c2f_run_stats;
c2f_status c2f_get_stats(const c2f_ctx* ctx, c2f_run_stats* out);

/* Serving (continuous batching).  c2f_submit validates a request and queues
 * it; serving lanes (each a HIP stream with its own work slots) take
 * requests from the head of the queue in arrival order and run them as one
 * fused launch, so that batches on different lanes overlap on the device.
 * A request is admitted when the device memory its lane must add (arrival
 * planes, work lists, output staging) fits within the context's budget
 * (hbm_budget_bytes of c2f_create, else 90 % of the memory free at
 * creation) next to what is already held; otherwise it waits for running
 * batches to finish, and idle lanes release their buffers.  A request that
 * does not fit even alone runs alone with fewer resident work slots, or
 * fails with ENOMEM.  Results are identical to c2f_simulate of the same
 * request.  Output pointers (host or device) must stay valid until the
 * request completes; device outputs are written on the lane's stream and
 * are complete when c2f_wait returns.  A landscape or weather set used by a
 * queued or running request cannot be unloaded (EBUSY).
 * EBUSY from c2f_submit when max_queue (4096) requests are already waiting. */
c2f_status c2f_submit(c2f_ctx* ctx, const c2f_sim_params* params, const c2f_outputs* out,
                      uint64_t* ticket);
/* *done = 1 once the request has completed (successfully or not). */
c2f_status c2f_poll(c2f_ctx* ctx, uint64_t ticket, int32_t* done);
/* Block until the request completes; returns its status and forgets the
 * ticket (ESTATE for an unknown or already waited ticket). */
c2f_status c2f_wait(c2f_ctx* ctx, uint64_t ticket);

/* Timing of a completed request, host steady clock in ms since the context
 * was created: submitted, started on a lane, outputs delivered. */
typedef struct {
    double submit_ms, start_ms, done_ms;
    double kernel_ms;          /* propagation time of the batch it ran in */
    int32_t batch_requests;    /* requests in that batch */
    int32_t batch_reps;        /* replications in that batch */
    int32_t lane;              /* serving lane that ran it */
    int32_t status;            /* its c2f_status */
} c2f_ticket_info;
/* c2f_wait that also reports the request's timing (info may be NULL). */
c2f_status c2f_wait_info(c2f_ctx* ctx, uint64_t ticket, c2f_ticket_info* info);

/* Serving configuration, before the first c2f_submit (ESTATE after):
 * lanes (1..16, default 4) concurrent batches; max_batch_reps (default
 * 2048) replications fused into one batch (a batch also stops taking
 * requests at 512 MiB of host-bound outputs); max_batch_grid resident work
 * groups one batch may use (0 = all that fit the device); admit_bytes the
 * device bytes admission plans against (0 = keep the default; at most the
 * context's budget). */
c2f_status c2f_set_serving(c2f_ctx* ctx, int32_t lanes, int32_t max_batch_reps,
                           int32_t max_batch_grid, uint64_t admit_bytes);

/* Device memory the context holds now (landscapes, weather, work slots,
 * lists, staging) and the limit serving admission plans against. */
c2f_status c2f_get_memory(c2f_ctx* ctx, uint64_t* bytes_held, uint64_t* admit_limit);

#ifdef __cplusplus
}
#endif

#endif /* C2F_H */
