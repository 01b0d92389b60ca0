/*
 * Cell2Fire reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of the fire-growth
 * hot path of Cell2Fire (Pais et al., "Cell2Fire: A Cell Based Forest Fire
 * Growth Model"): FBP rate of spread per cell (Sections 2.3 and 3.7), the
 * elliptical directional rate of eq. (1), and the synchronous send/receive
 * message loop of Algorithm 1 stepped minute by minute (Sections 3.1 and
 * 3.4).  Only the test-suite, the smoke check and the benchmark's CPU
 * baseline may call it; the simulator library never does.  It shares no
 * code, header or table with the simulator.
 *
 * All entry points return 0 on success and a negative value on bad input.
 */
#ifndef CELL2FIRE_ORACLE_H
#define CELL2FIRE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The oracle's FBP coefficients (a, b, c, q, BUI0) of fuel code 1..18
 * (16 D-2, 17 M-3, 18 M-4), and its crown base height (m) and crown fuel
 * load (kg/m^2). */
int oracle_fuel_coefficients(int32_t fuel, double* out5);
int oracle_crown_coefficients(int32_t fuel, double* out2);

/* Horn 3x3 gradient numerators with edge replication (east, north). */
int oracle_horn(int32_t rows, int32_t cols, const int16_t* elev, int32_t* gx, int32_t* gn);

/* One FBP evaluation for a single fuel at explicit slope (percent) and
 * upslope azimuth (degrees clockwise from north).  out[0..9] =
 * HROS, BROS, FROS, LB, RAZ (deg), ISI, WSV, BE, RSI, WSE. */
int oracle_fbp_point(int32_t fuel, double ffmc, double bui, double ws_kmh, double wd_from_deg,
                     double slope_pct, double upslope_az_deg, double pc_pct, double curing_pct,
                     double* out);

/* The same with foliar moisture content and percent dead fir (percent),
 * and out[10..13] = surface fuel consumption (kg/m^2), crown fraction
 * burned, total fuel consumption (kg/m^2), head fire intensity (kW/m).
 * oracle_fbp_point takes FMC 97 and PDF 50. */
int oracle_fbp_point_ext(int32_t fuel, double ffmc, double bui, double ws_kmh, double wd_from_deg,
                         double slope_pct, double upslope_az_deg, double pc_pct, double curing_pct,
                         double fmc_pct, double pdf_pct, double* out);

/* Directional rates of eq. (1) on the 8 centre-to-centre axes
 * (E, NE, N, NW, W, SW, S, SE) for the given head/back/flank rates and RAZ. */
void oracle_axis_ros(double hros, double bros, double fros, double raz_deg, double* out8);

/* Per-cell FBP field for one (scenario, period, replication).  Any output
 * pointer may be NULL.  hros/bros/fros include the replication's noise
 * multiplier; x8 is the unquantised axis rate, xu8 = x8 + u (the value that is
 * floored) and q8 the integer axis rate.  raz is in degrees. */
int oracle_eval_ros(int32_t rows, int32_t cols, int32_t cell_m, const uint8_t* fuel,
                    const int16_t* elev, double pc_pct, double curing_pct,
                    int32_t n_scen, int32_t n_wperiods, const float* weather,
                    int32_t scenario, int32_t period, int32_t rep, uint64_t seed, double sigma,
                    int32_t rounding, double* hros, double* bros, double* fros, double* lb,
                    double* raz, double* x8, double* xu8, int32_t* q8);

/* The same for the listed grid cells only: outputs are indexed by the
 * position in `cells` ([n_cells], [n_cells][8]); cells == NULL means every
 * cell in row-major order.  fmc_pct and pdf_pct as in oracle_fbp_point_ext;
 * cfb is the crown fraction burned and hfi the head fire intensity (kW/m,
 * with the rep's noise multiplier on the rate).  oracle_eval_ros takes FMC
 * 97 and PDF 50. */
int oracle_eval_ros_cells(int32_t rows, int32_t cols, int32_t cell_m, const uint8_t* fuel,
                          const int16_t* elev, double pc_pct, double curing_pct, double fmc_pct,
                          double pdf_pct, int32_t n_scen, int32_t n_wperiods, const float* weather,
                          int32_t scenario, int32_t period, int32_t rep, uint64_t seed, double sigma,
                          int32_t rounding, int64_t n_cells, const int32_t* cells, double* hros,
                          double* bros, double* fros, double* lb, double* raz, double* x8, double* xu8,
                          int32_t* q8, double* cfb, double* hfi);

/* Monte-Carlo fire simulation.  Replication r uses global index
 * rep_offset + r in every random draw.  Outputs may be NULL.
 * scar/arrival_* are [reps][rows*cols]; burn_count [rows*cols] is
 * overwritten; burned_cells, ignition_cell, scenario_out are [reps].
 * n_override entries (rep, period, cell) -> q[8] replace computed integer
 * axis rates (data only; used to replay another implementation's rounding).
 * stats (may be NULL) receives [ignitions, burning-cell-minutes, fbp evals,
 * burning-cell-periods, axis reach events]: a burning-cell-period is a
 * (replication, cell, period) whose rates the cell takes while burning
 * with at least one axis still leading to an available neighbour; an axis
 * reach event is progress along an axis reaching the neighbour's centre. */
int oracle_simulate(int32_t rows, int32_t cols, int32_t cell_m, const uint8_t* fuel,
                    const int16_t* elev, double pc_pct, double curing_pct,
                    int32_t n_scen, int32_t n_wperiods, int32_t period_min, const float* weather,
                    int32_t reps, int32_t rep_offset, int32_t n_periods, uint64_t seed,
                    double sigma, double threshold, int32_t rounding,
                    int32_t ignition_mode, int32_t ignition_cell,
                    int32_t scenario_mode, int32_t scenario_fixed,
                    int32_t n_override, const int32_t* override_key, const int32_t* override_q,
                    uint8_t* scar, int32_t* arrival_period, int32_t* arrival_minute,
                    uint32_t* burn_count, int64_t* burned_cells, int32_t* ignition_out,
                    int32_t* scenario_out, int64_t* stats);

/* oracle_simulate with the FBP landscape inputs and the ignition, burning-
 * window and burn-out options (oracle_simulate takes FMC 97, PDF 50 and
 * none of the options): fmc_pct and pdf_pct as in oracle_fbp_point_ext;
 * ignition_mode 3 draws the ignition cell with probability proportional to
 * ignition_weights[rows*cols] (integer weights); the ignition takes minute
 * ignition_period * period_min (0 <= ignition_period < n_periods, nothing
 * burns before); burn_hours in 1..24 limits spread and ignition to the first
 * burn_hours hours of every day counted from the start (0 = no limit);
 * burnout_ros > 0 (m/min) burns a cell out when, at an evaluation of its
 * rates for a period, its integer axis rates toward every in-grid burnable
 * neighbour are below it (assumption A5 (i)): it spreads no further;
 * hfi_min > 0 (kW/m) does the same when, at such an evaluation, the cell's
 * head fire intensity (with the noise multiplier on its rate) is below it
 * (assumption A5 (iv)).
 * ignition_mode 4 takes the ignition-point list of Section 3.2 (iii):
 * ignition_list holds n_ignitions (cell, period) pairs (0 <= period <
 * n_periods, any order; entries of one period keep theirs).  The cell of a
 * pair is lit at minute period * period_min, as a single ignition would be,
 * if it has fuel and has not burned yet (a reached cell waiting on the
 * threshold included); ignition_out reports the cell of the earliest entry.
 * ignition_period is unused in that mode. */
int oracle_simulate_ext(int32_t rows, int32_t cols, int32_t cell_m, const uint8_t* fuel,
                        const int16_t* elev, double pc_pct, double curing_pct, double fmc_pct,
                        double pdf_pct, int32_t n_scen, int32_t n_wperiods, int32_t period_min,
                        const float* weather, int32_t reps, int32_t rep_offset, int32_t n_periods,
                        uint64_t seed, double sigma, double threshold, int32_t rounding,
                        int32_t ignition_mode, int32_t ignition_cell, const uint32_t* ignition_weights,
                        int32_t ignition_period, int32_t burn_hours, double burnout_ros, double hfi_min,
                        int32_t n_ignitions, const int32_t* ignition_list,
                        int32_t scenario_mode, int32_t scenario_fixed,
                        int32_t n_override, const int32_t* override_key, const int32_t* override_q,
                        uint8_t* scar, int32_t* arrival_period, int32_t* arrival_minute,
                        uint32_t* burn_count, int64_t* burned_cells, int32_t* ignition_out,
                        int32_t* scenario_out, int64_t* stats);

/* Scar comparison (Section 4): per period t = 1..n_periods, the simulated
 * scar {arrival_minute in [0, t period_min]} against reference[t-1][n_cells]
 * (0-1): mse[t-1], ssim[t-1] (global SSIM, C1 = 1e-4, C2 = 9e-4, N - 1
 * normalisation), and delta_norm = Frobenius norm of the difference at the
 * last period.  Outputs may be NULL. */
int oracle_scar_metrics(int64_t n_cells, int32_t n_periods, int32_t period_min, const int32_t* arrival_minute,
                        const uint8_t* reference, double* mse, double* ssim, double* delta_norm);

#ifdef __cplusplus
}
#endif
#endif
