// Landscape and weather preparation, and the per-cell FBP field kernel.
//
//  * cell records: fuel, burnable-neighbour mask, Horn slope numerators and
//    the FBP slope factor of every cell (Section 3.3 (i)-(ii));
//  * burnable-cell list (row-major) and the burnable cell nearest the centre
//    (ignition choices of Section 3.1, uncertainty source (1));
//  * weather table: per (scenario, period) FBP terms that do not depend on
//    the cell (Section 3.5 (iv));
//  * eval_ros: the per-cell rates of one (scenario, period, rep).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"
#include "kernels.h"
#include "types.h"

namespace c2f {

// ------------------------------------------------------------ utilities
__global__ void fill_u32_kernel(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int fill_grid(size_t n) {
    size_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// -------------------------------------------------- landscape preparation

// Cell records.  Horn's 3x3 gradient numerators with replicated edges:
// gx = east column - west column (weights 1,2,1), gn = north row - south row.
// grad_from (may be NULL): take the Horn numerators from these records (a
// landscape derived from another with the same elevation) instead of elev.
__global__ void cellrec_kernel(const uint8_t* __restrict__ fuel, const int16_t* __restrict__ elev,
                               const CellRec* __restrict__ grad_from, int rows, int cols, double cell_m,
                               CellRec* __restrict__ recs, int32_t* __restrict__ overflow) {
    const size_t n = (size_t)rows * cols;
    const int DR[8] = {0, -1, -1, -1, 0, 1, 1, 1};
    const int DC[8] = {1, 1, 0, -1, -1, -1, 0, 1};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / cols), c = (int)(i - (size_t)r * cols);
        uint32_t mask = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int rr = r + DR[k], cc = c + DC[k];
            if (rr >= 0 && rr < rows && cc >= 0 && cc < cols && fuel[(size_t)rr * cols + cc] != 0) mask |= 1u << k;
        }
        int gx = 0, gn = 0;
        if (grad_from) {
            const uint32_t g = grad_from[i].grad;
            gx = (int)(int16_t)(g & 0xFFFFu);
            gn = (int)(int16_t)(g >> 16);
        } else if (elev) {
            const int rn = r > 0 ? r - 1 : 0, rs = r < rows - 1 ? r + 1 : rows - 1;
            const int cw = c > 0 ? c - 1 : 0, ce = c < cols - 1 ? c + 1 : cols - 1;
            auto z = [&](int rr, int cc) { return (int)elev[(size_t)rr * cols + cc]; };
            gx = (z(rn, ce) + 2 * z(r, ce) + z(rs, ce)) - (z(rn, cw) + 2 * z(r, cw) + z(rs, cw));
            gn = (z(rn, cw) + 2 * z(rn, c) + z(rn, ce)) - (z(rs, cw) + 2 * z(rs, c) + z(rs, ce));
            if (gx > 32767 || gx < -32767 || gn > 32767 || gn < -32767) {
                atomicOr(overflow, 1);
                gx = gn = 0;
            }
        }
        CellRec rec;
        const int f = fuel[i];
        rec.info = (uint32_t)f | (mask << 8);
        rec.grad = (uint32_t)(uint16_t)(int16_t)gx | ((uint32_t)(uint16_t)(int16_t)gn << 16);
        rec.pad[0] = rec.pad[1] = 0u;
        rec.sfc = 1.0;
        rec.sfd = 1.0;
        if ((gx | gn) != 0 && f != kNonFuel) {
            // SF^(1/c) of the rate curve(s) the cell's slope effect uses
            const double sf = slope_factor(gx, gn, cell_m);
            // mixedwoods: their conifer curve (C-2 for M-1/M-2, their own
            // dead-fir curve for M-3/M-4) and the D-1 curve
            const bool mix_pc = (f == kM1 || f == kM2), mixed = mix_pc || f == kM3 || f == kM4;
            rec.sfc = pow(sf, 1.0 / kCoef64[mix_pc ? kC2 : f].c);
            if (mixed) rec.sfd = pow(sf, 1.0 / kCoef64[kD1].c);
        }
        recs[i] = rec;
    }
}

// Burnable-cell list in row-major order: per-tile counts, one-block scan,
// ordered scatter.  A tile is kTile consecutive cells handled by one block.
constexpr int kTileThreads = 256;
constexpr int kTile = kTileThreads * 16;

__global__ void burnable_count_kernel(const uint8_t* __restrict__ fuel, int64_t n,
                                      int32_t* __restrict__ tile_counts) {
    __shared__ int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    int local = 0;
    for (int k = threadIdx.x; k < kTile; k += kTileThreads) {
        const int64_t i = t0 + k;
        local += (i < n && fuel[i] != 0);
    }
    atomicAdd(&s_cnt, local);
    __syncthreads();
    if (threadIdx.x == 0) tile_counts[blockIdx.x] = s_cnt;
}

__global__ void burnable_scan_kernel(int32_t* __restrict__ tile_counts, int n_tiles, LandDev* land) {
    // single block of 1024 threads: exclusive scan in place
    __shared__ int s_part[1024];
    const int per = (n_tiles + 1023) / 1024;
    const int b = threadIdx.x * per;
    int sum = 0;
    for (int k = 0; k < per && b + k < n_tiles; ++k) sum += tile_counts[b + k];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = (threadIdx.x >= (unsigned)off) ? s_part[threadIdx.x - off] : 0;
        __syncthreads();
        s_part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = s_part[threadIdx.x] - sum;   // exclusive prefix of this thread's range
    for (int k = 0; k < per && b + k < n_tiles; ++k) {
        const int c = tile_counts[b + k];
        tile_counts[b + k] = run;
        run += c;
    }
    if (threadIdx.x == 1023) land->n_burnable = s_part[1023];
}

__global__ void burnable_scatter_kernel(const uint8_t* __restrict__ fuel, int64_t n,
                                        const int32_t* __restrict__ tile_offsets,
                                        int32_t* __restrict__ list) {
    __shared__ int s_wave[kTileThreads / 64];
    __shared__ int s_base;
    if (threadIdx.x == 0) s_base = tile_offsets[blockIdx.x];
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k0 = 0; k0 < kTile; k0 += kTileThreads) {
        const int64_t i = t0 + k0 + threadIdx.x;
        const bool b = (i < n) && fuel[i] != 0;
        const uint64_t m = __ballot(b);
        if (lane == 0) s_wave[wave] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < kTileThreads / 64; ++w) {
            if (w < wave) before += s_wave[w];
            total += s_wave[w];
        }
        if (b) {
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            list[s_base + before + rank] = (int32_t)i;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_base += total;
        __syncthreads();
    }
}

// Burnable cell nearest to (rows/2, cols/2); ties go to the lower index.
// Keys (d^2 << 32 | index) are reduced within each wave before one atomic.
__global__ void centre_kernel(const uint8_t* __restrict__ fuel, int rows, int cols, LandDev* land) {
    const size_t n = (size_t)rows * cols;
    const int cr = rows / 2, cc = cols / 2;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = (size_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        const size_t i = base + threadIdx.x;
        unsigned long long key = ~0ull;
        if (i < n && fuel[i] != 0) {
            const long long dr = (long long)(i / cols) - cr, dc = (long long)(i % cols) - cc;
            key = ((unsigned long long)(dr * dr + dc * dc) << 32) | (unsigned long long)i;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(key, off);
            key = o < key ? o : key;
        }
        if ((threadIdx.x & 63) == 0 && key != ~0ull) atomicMin(&land->centre_key, key);
    }
}

// Landscape constants: M-1/M-2 conifer fraction and the O-1 curing factor
// (0.005 (exp(0.061 C) - 1) below 58.8 % curing, 0.176 + 0.02 (C - 58.8)
// above); M-3/M-4 dead-fir fraction; from the foliar moisture content FMC the
// C-6 moisture effect FME = 1000 (1.5 - 0.00275 FMC)^4 / (460 + 25.9 FMC)
// over its average 0.778, and the critical surface intensity for crowning
// 0.001 CBH^1.5 (460 + 25.9 FMC)^1.5 of every fuel.
__global__ void fbpconst_kernel(LandDev* land, float fmc_f, float pdf_f) {
    const int f = threadIdx.x;
    const double fmc = (double)fmc_f;
    const double h = pow(460.0 + 25.9 * fmc, 1.5);
    if (f < kNumFuels) {
        const double csi = 0.001 * pow(kCrown[f].cbh, 1.5) * h;
        land->csi64[f] = csi;
        land->csi32[f] = (float)csi;
    }
    if (f == 0) {
        const double fme = 1000.0 * pow(1.5 - 0.00275 * fmc, 4.0) / (460.0 + 25.9 * fmc);
        land->pdf_w64 = (double)pdf_f / 100.0;
        land->fme_r64 = fme / 0.778;
        land->pdf_w32 = pdf_f / 100.0f;
        land->fme_r32 = (float)(fme / 0.778);
    }
}

hipError_t launch_fbp_consts(LandDev* land, float fmc, float pdf, hipStream_t s) {
    hipLaunchKernelGGL(fbpconst_kernel, dim3(1), dim3(64), 0, s, land, fmc, pdf);
    return hipGetLastError();
}

__global__ void landconst_kernel(LandDev* land, float pc, float curing, int cell_m) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double c = (double)curing;
    land->pc_w64 = (double)pc / 100.0;
    land->cf64 = (c < 58.8) ? 0.005 * (exp(0.061 * c) - 1.0) : 0.176 + 0.02 * (c - 58.8);
    land->cell_m64 = (double)cell_m;
    const float cf = curing;
    land->pc_w32 = pc / 100.0f;
    land->cf32 = (cf < 58.8f) ? 0.005f * (expf(0.061f * cf) - 1.0f) : 0.176f + 0.02f * (cf - 58.8f);
    land->cell_m32 = (float)cell_m;
    const unsigned long long key = land->centre_key;
    land->centre_cell = (key == ~0ull) ? -1 : (int32_t)(key & 0xFFFFFFFFull);
}

hipError_t launch_prepare_landscape(const uint8_t* fuel, const int16_t* elev, const CellRec* grad_from,
                                    int rows, int cols, int cell_m, float pc, float curing, float fmc,
                                    float pdf, CellRec* recs, int32_t* burnable, int32_t* tile_scratch,
                                    LandDev* land, hipStream_t s) {
    const int64_t n = (int64_t)rows * cols;
    const int g = fill_grid((size_t)n);
    hipError_t e;
    // LandDev: zero, then centre key = max
    if ((e = launch_fill_u32((uint32_t*)land, sizeof(LandDev) / 4, 0u, s)) != hipSuccess) return e;
    if ((e = launch_fill_u32((uint32_t*)&land->centre_key, 2, 0xFFFFFFFFu, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(cellrec_kernel, dim3(g), dim3(256), 0, s, fuel, elev, grad_from, rows, cols,
                       (double)cell_m, recs, &land->grad_overflow);
    const int n_tiles = (int)((n + kTile - 1) / kTile);
    hipLaunchKernelGGL(burnable_count_kernel, dim3(n_tiles), dim3(kTileThreads), 0, s, fuel, n, tile_scratch);
    hipLaunchKernelGGL(burnable_scan_kernel, dim3(1), dim3(1024), 0, s, tile_scratch, n_tiles, land);
    hipLaunchKernelGGL(burnable_scatter_kernel, dim3(n_tiles), dim3(kTileThreads), 0, s, fuel, n, tile_scratch, burnable);
    hipLaunchKernelGGL(centre_kernel, dim3(g), dim3(256), 0, s, fuel, rows, cols, land);
    hipLaunchKernelGGL(landconst_kernel, dim3(1), dim3(64), 0, s, land, pc, curing, cell_m);
    hipLaunchKernelGGL(fbpconst_kernel, dim3(1), dim3(64), 0, s, land, fmc, pdf);
    return hipGetLastError();
}

int64_t tile_scratch_entries(int64_t n_cells) { return (n_cells + kTile - 1) / kTile; }

// fuel[cells[k]] = codes[k]: the edits of a derived landscape (cells are
// checked on the host).
__global__ void fuel_edit_kernel(uint8_t* __restrict__ fuel, const int32_t* __restrict__ cells,
                                 const uint8_t* __restrict__ codes, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) fuel[cells[k]] = codes[k];
}

hipError_t launch_fuel_edits(uint8_t* fuel, const int32_t* cells, const uint8_t* codes, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fuel_edit_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fuel, cells, codes, n);
    return hipGetLastError();
}

// ------------------------------------------------------- weather table

template <typename R>
__global__ void weather_table_kernel(const float* __restrict__ wx, int n_rows, R* __restrict__ table) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    const float* w = wx + (size_t)i * 4;
    R row[kRowLen];
    weather_row<R>(coef_table<R>(), w[0], w[1], w[2], w[3], row);
    for (int k = 0; k < kRowLen; ++k) table[(size_t)i * kRowLen + k] = row[k];
}

hipError_t launch_weather_table(const float* wx, int n_rows, double* t64, float* t32, hipStream_t s) {
    const int g = (n_rows + 127) / 128;
    hipLaunchKernelGGL(weather_table_kernel<double>, dim3(g), dim3(128), 0, s, wx, n_rows, t64);
    hipLaunchKernelGGL(weather_table_kernel<float>, dim3(g), dim3(128), 0, s, wx, n_rows, t32);
    return hipGetLastError();
}

// ------------------------------------------------------------- eval_ros

template <typename R>
__global__ void eval_ros_kernel(EvalArgs a) {
    RateCtx<R> X;
    X.coef = coef_table<R>();
    X.coef64 = coef_table<double>();
    X.L = land_consts<R>(a.land);
    X.L64 = land_consts<double>(a.land);
    X.rows = (const R*)a.table + (size_t)a.scenario * a.n_wp * kRowLen;
    X.rows64 = a.table64 + (size_t)a.scenario * a.n_wp * kRowLen;
    X.row_stride = kRowLen;
    X.coef32 = coef_table<float>();
    X.L32 = land_consts<float>(a.land);
    X.rows32 = a.table32 ? a.table32 + (size_t)a.scenario * a.n_wp * kRowLen : nullptr;
    X.seed = a.seed;
    X.sigma = (R)a.sigma;
    X.rounding = a.rounding;
    X.rep = a.rep;
    X.burnout = 0.f;
    X.hfi_min = 0.f;
    const size_t ro = (size_t)a.period * kRowLen;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n_cells; i += gridDim.x * blockDim.x) {
        const CellRec rec = a.cells[i];
        const int f = rec_fuel(rec.info);
        if (f == 0) {
            if (a.hros) a.hros[i] = 0;
            if (a.bros) a.bros[i] = 0;
            if (a.fros) a.fros[i] = 0;
            if (a.lb) a.lb[i] = 0;
            if (a.raz) a.raz[i] = 0;
            if (a.cfb) a.cfb[i] = 0;
            if (a.hfi) a.hfi[i] = 0;
            for (int k = 0; k < 8; ++k) {
                if (a.x8) a.x8[(size_t)i * 8 + k] = 0;
                if (a.q8) a.q8[(size_t)i * 8 + k] = 0;
            }
            continue;
        }
        const CellRates<R> cr = cell_rates<R>(X.coef, X.coef64, rec, X.rows + ro, X.rows64 + ro, X.L, X.L64);
        const R mu = noise_mult<R>(a.seed, (uint32_t)i, (uint32_t)a.period, a.rep, (R)a.sigma);
        R x[8];
        axis_rates<R>(cr, mu, x);
        int32_t q[8];
        axis_q<R>(X, rec, (uint32_t)i, (uint32_t)a.period, q);
        if (a.hros) a.hros[i] = (double)(cr.h * mu);
        if (a.bros) a.bros[i] = (double)(cr.b * mu);
        if (a.fros) a.fros[i] = (double)((cr.h + cr.b) / ((R)2 * cr.lb) * mu);
        if (a.lb) a.lb[i] = (double)cr.lb;
        if (a.cfb || a.hfi) {
            R cfb = (R)0;
            const R hfi = head_intensity<R>(cr, f, X.rows + ro, X.L, &cfb) * mu;
            if (a.cfb) a.cfb[i] = (double)cfb;
            if (a.hfi) a.hfi[i] = (double)hfi;
        }
        if (a.raz) {
            double az = 0.0;
            if (cr.wsv > (R)0) {
                az = (double)m_atan2(cr.wx, cr.wy) * (180.0 / 3.14159265358979323846);
                if (az < 0.0) az += 360.0;
            }
            a.raz[i] = az;
        }
        for (int k = 0; k < 8; ++k) {
            if (a.x8) a.x8[(size_t)i * 8 + k] = (double)x[k];
            if (a.q8) a.q8[(size_t)i * 8 + k] = q[k];
        }
    }
}

hipError_t launch_eval_ros(int precision, const EvalArgs& a, hipStream_t s) {
    const int g = fill_grid((size_t)a.n_cells);
    if (precision == 1) hipLaunchKernelGGL(eval_ros_kernel<float>, dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(eval_ros_kernel<double>, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace c2f
