// Device building blocks: Philox4x32-10, per-period weather terms, the FBP
// rate evaluation of one cell, and the directional rates of eq. (1).
// Everything is templated on the arithmetic type R (double or float).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fuel_table.h"
#include "ln64.h"
#include "types.h"

namespace c2f {

// ------------------------------------------------------------------ math
// Explicit precision dispatch so float code never widens to double.
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
__device__ __forceinline__ double m_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float m_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double m_log(double x) { return ln_f64(x); }
__device__ __forceinline__ float m_log(float x) { return logf(x); }
__device__ __forceinline__ double m_pow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float m_pow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_sin(double x) { return sin(x); }
__device__ __forceinline__ float m_sin(float x) { return sinf(x); }
__device__ __forceinline__ double m_cos(double x) { return cos(x); }
__device__ __forceinline__ float m_cos(float x) { return cosf(x); }
__device__ __forceinline__ double m_floor(double x) { return floor(x); }
__device__ __forceinline__ float m_floor(float x) { return floorf(x); }
__device__ __forceinline__ double m_atan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float m_atan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double m_fmod(double x, double y) { return fmod(x, y); }
__device__ __forceinline__ float m_fmod(float x, float y) { return fmodf(x, y); }

// Reciprocals: v_rcp_f32 (1 ulp) for FP32; v_rcp_f64 refined by two Newton
// steps for FP64 (about 1 ulp).  a * recip(b) replaces the long
// correctly-rounded division sequences on the rate path.
__device__ __forceinline__ float recip(float b) { return __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double recip(double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    r = fma(fma(-b, r, 1.0), r, r);
    return r;
}

// Powers on the rate path: x >= 0 (a rate-curve base, 1 - exp(-0.03 WSV),
// or a wind speed) and y a positive fuel constant below 5, as exp(y ln x).
// A relative error of about one ulp in ln x becomes an absolute error of
// |y ln x| ulp in the exponent, so the result keeps a relative error of a
// few ulp for these bases, at a third of the instructions of the general
// pow() (which rounds exactly and handles every special case).  FP32 uses
// the hardware base-2 logarithm and exponential.  x = 0 gives 0.
__device__ __forceinline__ double rate_pow(double x, double y) { return exp(y * ln_f64(x)); }
__device__ __forceinline__ float rate_pow(float x, float y) { return exp2f(y * log2f(x)); }

// cos(2 pi u) for the Box-Muller draw, without a general argument reduction.
__device__ __forceinline__ double cos_2pi(double u) { return cospi(2.0 * u); }
__device__ __forceinline__ float cos_2pi(float u) { return cospif(2.0f * u); }

// ln(1 - x) for 0 <= x <= 0.99 in FP32 from one logarithm: with u = 1 - x
// rounded, ln(u) x / (1 - u) corrects the rounding of u (the log1p form of
// Goldberg, 1991; 1 - u is exact here), so a small x keeps its full
// relative precision.
__device__ __forceinline__ float log_1m(float x) {
    const float u = 1.0f - x;
    if (u == 1.0f) return -x;
    return logf(u) * (x * __builtin_amdgcn_rcpf(1.0f - u));
}

template <typename R> struct Const;
template <> struct Const<double> { static constexpr double pi = 3.14159265358979323846; };
template <> struct Const<float> { static constexpr float pi = 3.14159265358979323846f; };

// --------------------------------------------------------------- Philox
// Philox4x32-10 block function (Salmon et al., SC'11): ten rounds of two
// 32x32->64 multiplies, key bumped by the Weyl constants between rounds.
// Each product is formed once in 64 bits (one v_mad_u64_u32 instead of a
// low and a high multiply).
__device__ __forceinline__ uint4 philox4x32_10(uint4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x.z;
        x = make_uint4((uint32_t)(p1 >> 32) ^ x.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ x.w ^ k1,
                       (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x;
}

// Counter layout shared by every random draw: (cell, period, rep, tag).
// Tags: 0 ROS noise, 1-2 rounding uniforms for axes 0-3 / 4-7,
// 3 ignition cell, 4 weather scenario (per-rep draws use cell = period = ~0).
__device__ __forceinline__ uint4 draw(uint64_t seed, uint32_t cell, uint32_t period, uint32_t rep,
                                      uint32_t tag) {
    return philox4x32_10(make_uint4(cell, period, rep, tag), (uint32_t)seed, (uint32_t)(seed >> 32));
}

// 24-bit uniform in [0, 1) from the high bits of a 32-bit word (exact in float).
template <typename R>
__device__ __forceinline__ R unit24(uint32_t x) {
    return (R)(x >> 8) * (R)(1.0 / 16777216.0);
}

// ------------------------------------------------------- weather terms
// Per (scenario, period) quantities that do not depend on the cell; kept in
// a table computed once per weather upload.  Layout of one row:
//   [0] f(F)   [1] ISZ = 0.208 f(F)   [2] WS sin(WAZ)   [3] WS cos(WAZ)
//   [4 + f] BUI effect of fuel f      [23 + f] 1 - exp(-b_f ISZ) of pure fuel f
//   [42 + f] surface fuel consumption of fuel f

template <typename R>
struct CoefR {
    R a, b, c, q, bui0;
};

// Rate of spread of one unmixed fuel: a (1 - exp(-b ISI))^c.
template <typename R>
__device__ __forceinline__ R rsi_pure(const CoefR<R>& k, R isi) {
    return k.a * rate_pow(-m_expm1(-k.b * isi), k.c);
}

// Surface fuel consumption (kg/m^2) of an unmixed fuel from FFMC and BUI
// (M-1/M-2 mix the C-2 and D-1 values by percent conifer where they are
// used; they get 0 here).
template <typename R>
__device__ R surface_consumption(int f, R ffmc, R bui) {
    switch (f) {
        case kC1:
            return ffmc > (R)84 ? (R)0.75 + (R)0.75 * m_sqrt((R)1 - m_exp((R)-0.23 * (ffmc - (R)84)))
                                : (R)0.75 - (R)0.75 * m_sqrt((R)1 - m_exp((R)-0.23 * ((R)84 - ffmc)));
        case kC2:
        case kM3:
        case kM4: return (R)5 * ((R)1 - m_exp((R)-0.0115 * bui));
        case kC3:
        case kC4: return (R)5 * m_pow((R)1 - m_exp((R)-0.0164 * bui), (R)2.24);
        case kC5:
        case kC6: return (R)5 * m_pow((R)1 - m_exp((R)-0.0149 * bui), (R)2.48);
        case kC7: {
            const R ffc = ffmc > (R)70 ? (R)2 * ((R)1 - m_exp((R)-0.104 * (ffmc - (R)70))) : (R)0;
            return ffc + (R)1.5 * ((R)1 - m_exp((R)-0.0201 * bui));
        }
        case kD1:
        case kD2: return (R)1.5 * ((R)1 - m_exp((R)-0.0183 * bui));
        case kS1: return (R)4 * ((R)1 - m_exp((R)-0.025 * bui)) + (R)4 * ((R)1 - m_exp((R)-0.034 * bui));
        case kS2: return (R)10 * ((R)1 - m_exp((R)-0.013 * bui)) + (R)6 * ((R)1 - m_exp((R)-0.060 * bui));
        case kS3: return (R)12 * ((R)1 - m_exp((R)-0.0166 * bui)) + (R)20 * ((R)1 - m_exp((R)-0.0210 * bui));
        case kO1a:
        case kO1b: return (R)kGrassFuelLoad;
        default: return (R)0;
    }
}

// Fill one table row from FFMC, BUI, wind speed (km/h) and the azimuth the
// wind comes from.  The fire heads downwind: WAZ = WD + 180 degrees.
template <typename R>
__device__ void weather_row(const CoefR<R>* coef, float ffmc_f, float bui_f, float ws_f, float wd_f,
                            R* row) {
    const R ffmc = (R)ffmc_f, bui = (R)bui_f, ws = (R)ws_f, wd = (R)wd_f;
    const R m = (R)147.2 * ((R)101 - ffmc) / ((R)59.5 + ffmc);   // fine fuel moisture
    const R ff = (R)91.9 * m_exp((R)-0.1386 * m) * ((R)1 + m_pow(m, (R)5.31) / (R)4.93e7);
    const R isz = (R)0.208 * ff;
    const R waz = m_fmod(wd + (R)180, (R)360) * (Const<R>::pi / (R)180);
    row[0] = ff;
    row[1] = isz;
    row[2] = ws * m_sin(waz);
    row[3] = ws * m_cos(waz);
    for (int f = 0; f < kNumFuels; ++f) {
        const CoefR<R>& k = coef[f];
        R be = (R)1;
        if (f != kNonFuel && bui > (R)0)
            be = m_exp((R)50 * m_log(k.q) * ((R)1 / bui - (R)1 / k.bui0));
        row[kRowBE + f] = be;
        row[kRowG + f] = (k.a > (R)0) ? -m_expm1(-k.b * isz) : (R)0;
        row[kRowSFC + f] = surface_consumption<R>(f, ffmc, bui);
    }
    for (int k = kRowSFC + kNumFuels; k < kRowLen; ++k) row[k] = (R)0;
}

// ----------------------------------------------------------- cell rates
__device__ __forceinline__ int rec_fuel(uint32_t info) { return (int)(info & 0xFFu); }
__device__ __forceinline__ uint32_t rec_nbmask(uint32_t info) { return (info >> 8) & 0xFFu; }
__device__ __forceinline__ int rec_gx(uint32_t g) { return (int)(int16_t)(g & 0xFFFFu); }
__device__ __forceinline__ int rec_gn(uint32_t g) { return (int)(int16_t)(g >> 16); }

// Landscape-wide constants of the mixed, grass and crowning fuels.
template <typename R>
struct LandR {
    R pc_w;    // percent conifer / 100 (M-1, M-2)
    R cf;      // grass curing factor (O-1a, O-1b)
    R cell_m;  // cell width, metres
    R pdf_w;   // percent dead fir / 100 (M-3, M-4)
    R fme_r;   // C-6 foliar moisture effect / its average 0.778
    const R* csi;   // critical surface intensity for crowning per fuel, kW/m
};

__device__ __forceinline__ bool is_grass(int f) { return f == kO1a || f == kO1b; }
__device__ __forceinline__ bool is_mix_pc(int f) { return f == kM1 || f == kM2; }
__device__ __forceinline__ bool is_mix_pdf(int f) { return f == kM3 || f == kM4; }

template <typename R>
__device__ __forceinline__ R rsi_fuel(const CoefR<R>* coef, int f, R isi, const LandR<R>& L) {
    // Mixedwoods blend a conifer curve with D-1: M-1/M-2 the C-2 curve by
    // percent conifer, M-3/M-4 their dead-fir curve by percent dead fir
    // (M-2 and M-4 take 0.2 of D-1).  Every lane evaluates its own (or the
    // C-2) curve, and the D-1 curve only runs when some lane of the wave is
    // a mixedwood.
    const bool mix_pc = is_mix_pc(f), mixed = mix_pc || is_mix_pdf(f);
    R r = rsi_pure(coef[mix_pc ? (int)kC2 : f], isi);
    if (__any(mixed)) {
        const R d1 = rsi_pure(coef[kD1], isi);
        if (mixed) {
            const R w = mix_pc ? L.pc_w : L.pdf_w;
            const R wd1 = (f == kM2 || f == kM4) ? (R)0.2 * ((R)1 - w) : ((R)1 - w);
            r = w * r + wd1 * d1;
        }
    }
    return is_grass(f) ? r * L.cf : r;
}

// Slope-equivalent wind speed (km/h).  The slope-adjusted zero-wind rate
// RSF = SF x RSZ inverted on the fuel's rate curve gives ISF = ln(1 - (RSF /
// (CF a))^(1/c)) / -b with the curve's 0.01 floor inside the logarithm.
// Because RSZ = CF a (1 - exp(-b ISZ))^c, (RSF / (CF a))^(1/c) is exactly
// SF^(1/c) (1 - exp(-b ISZ)): sfc/sfd carry SF^(1/c) per cell and the row
// carries 1 - exp(-b ISZ) per fuel.  Mixedwood takes the percent-conifer
// weighted ISF of the C-2 and D-1 curves.
__device__ __forceinline__ double isf_curve(const CoefR<double>& k, double sfc, double g) {
    double t = 1.0 - sfc * g;
    if (t < 0.01) t = 0.01;
    return -ln_f64(t) * recip(k.b);
}

__device__ __forceinline__ double slope_wind(const CoefR<double>* coef, int f, double sfc, double sfd,
                                          const double* row, const LandR<double>& L) {
    const double ff = row[0], isz = row[1];
    // every lane inverts its own (or the C-2) curve; the D-1 curve only runs
    // when some lane of the wave is mixedwood
    const bool mix_pc = is_mix_pc(f), mixed = mix_pc || is_mix_pdf(f);
    const int fa = mix_pc ? (int)kC2 : f;
    double isf = isf_curve(coef[fa], sfc, row[kRowG + fa]);
    if (__any(mixed)) {
        const double d1 = isf_curve(coef[kD1], sfd, row[kRowG + kD1]);
        if (mixed) {
            const double w = mix_pc ? L.pc_w : L.pdf_w;
            isf = w * isf + (1.0 - w) * d1;
        }
    }
    double wse = ln_f64(isf * recip(isz)) * (1.0 / 0.05039);
    if (wse > 40.0) {
        wse = (isf < 0.999 * 2.496 * ff) ? 28.0 - ln_f64(1.0 - isf * recip(2.496 * ff)) * (1.0 / 0.0818) : 112.45;
    }
    return wse;
}

// The same in FP32 for the ordinary branch (WSE <= 40 km/h).  ln(1 - x) is
// taken with log1p accuracy (log_1m), so a gentle slope (x close to the zero-slope value)
// keeps full relative precision in ISF, and WSE = ln(ISF / ISZ) / 0.05039
// then carries an absolute error of a few 1e-6 km/h.  Near and above the
// 40 km/h branch point the caller switches to slope_wind in FP64, and so it
// does where ill is set: x = SF^(1/c) (1 - exp(-b ISZ)) above 0.8, where
// ln(1 - x) multiplies the relative error of x by x / (1 - x) and the 0.01
// floor of the curve is near (steep slopes in fast fuels).
constexpr float kIllX = 0.8f;

__device__ __forceinline__ float isf_curve32(const CoefR<float>& k, float x) {
    return -log_1m(x > 0.99f ? 0.99f : x) * recip(k.b);
}

__device__ __forceinline__ float slope_wind32(const CoefR<float>* coef, int f, float sfc, float sfd,
                                              const float* row, const LandR<float>& L, bool& ill) {
    const bool mix_pc = is_mix_pc(f), mixed = mix_pc || is_mix_pdf(f);
    const int fa = mix_pc ? (int)kC2 : f;
    const float xo = sfc * row[kRowG + fa];
    float isf = isf_curve32(coef[fa], xo);
    ill = xo > kIllX;
    if (__any(mixed)) {
        const float xd = sfd * row[kRowG + kD1];
        const float d1 = isf_curve32(coef[kD1], xd);
        if (mixed) {
            const float w = mix_pc ? L.pc_w : L.pdf_w;
            isf = w * isf + (1.0f - w) * d1;
            ill = ill || xd > kIllX;
        }
    }
    return m_log(isf * recip(row[1])) * (1.0f / 0.05039f);
}

// Head and back rates, length-to-breadth ratio and the effective wind
// vector (east, north components; its direction is the head direction).
template <typename R>
struct CellRates {
    R h, b, lb, lbm1, wx, wy, wsv;   // lbm1 = LB - 1, kept separately for accuracy
    R rss;                           // C-6: its surface head rate; other fuels: h
    // WSV lies within kEdgeWsv km/h of a speed where the model switches
    // form and its value jumps: f(W) at 40 km/h, grass LB at 1 km/h.  An
    // FP32 evaluation there may take the other branch than FP64.
    bool edge;
};

constexpr float kEdgeWsv = 1e-3f;

// C-6 crown fire: the surface rate rss at spread index isi becomes rss +
// CFB (RSC - rss), RSC = 60 (1 - exp(-0.0497 ISI)) FME / 0.778 and CFB =
// 1 - exp(-0.23 (rss - RSO)) above the critical surface rate RSO = CSI /
// (300 SFC), 0 below it.
template <typename R>
__device__ __forceinline__ R c6_rate(R rss, R isi, R rso, R fme_r) {
    const R cfb = rss > rso ? -m_expm1((R)-0.23 * (rss - rso)) : (R)0;
    return rss + cfb * ((R)60 * -m_expm1((R)-0.0497 * isi) * fme_r - rss);
}

// Everything is evaluated in R.  In FP32 the slope-equivalent wind switches
// to FP64 from 39 km/h up: inverting the rate curve near its asymptote (the
// WSE > 40 branch) turns a relative error of 1e-7 in ISF into ~1e-4 in WSE.
// It does so too where the inversion's argument is ill-conditioned
// (slope_wind32's ill).
// row64 is the FP64 weather row of the same (scenario, period).
template <typename R>
__device__ __forceinline__ CellRates<R> cell_rates(const CoefR<R>* coef, const CoefR<double>* coef64,
                                                const CellRec& rec, const R* row, const double* row64,
                                                const LandR<R>& L, const LandR<double>& L64) {
    const int f = rec_fuel(rec.info), gx = rec_gx(rec.grad), gn = rec_gn(rec.grad);
    R wx = row[2], wy = row[3];
    if ((gx | gn) != 0) {
        R wse = (R)0;
        bool need64 = true;
        if constexpr (sizeof(R) == 4) {
            bool ill;
            wse = slope_wind32(coef, f, (float)rec.sfc, (float)rec.sfd, row, L, ill);
            need64 = ill || !(wse < 39.0f);
        }
        if (need64) wse = (R)slope_wind(coef64, f, rec.sfc, rec.sfd, row64, L64);
        const R ig = recip(m_sqrt((R)gx * (R)gx + (R)gn * (R)gn));
        wx += wse * ((R)gx * ig);                                          // along the upslope unit vector
        wy += wse * ((R)gn * ig);
    }
    const R wsv = m_sqrt(wx * wx + wy * wy);
    // exp(0.05039 WSV) is f(W) up to 40 km/h, and its reciprocal is the back
    // fire's wind function at every speed
    const R ew = m_exp((R)0.05039 * wsv);
    const R fw = (wsv <= (R)40) ? ew : (R)12 * -m_expm1((R)-0.0818 * (wsv - (R)28));
    const R be = row[kRowBE + f];
    const R isz = row[1];
    CellRates<R> out;
    const R isi_h = isz * fw, isi_b = isz * recip(ew);
    out.h = rsi_fuel(coef, f, isi_h, L) * be;
    out.b = rsi_fuel(coef, f, isi_b, L) * be;
    out.rss = out.h;
    if (__any(f == kC6)) {
        if (f == kC6) {
            const R sfc = row[kRowSFC + kC6];
            const R rso = sfc > (R)0 ? L.csi[kC6] * recip((R)300 * sfc) : (R)3.0e38;
            out.h = c6_rate<R>(out.rss, isi_h, rso, L.fme_r);
            out.b = c6_rate<R>(out.b, isi_b, rso, L.fme_r);
        }
    }
    // LB - 1: grass 1.1 WSV^0.464 - 1 (0 below 1 km/h), other fuels
    // 8.729 (1 - exp(-0.030 WSV))^2.155, as one power per lane
    const bool grass = is_grass(f);
    const R lbase = grass ? wsv : -m_expm1((R)-0.030 * wsv);
    const R lpow = rate_pow(lbase, grass ? (R)0.464 : (R)2.155);
    out.lbm1 = grass ? ((wsv >= (R)1) ? (R)1.1 * lpow - (R)1 : (R)0) : (R)8.729 * lpow;
    out.lb = (R)1 + out.lbm1;
    out.wx = wx;
    out.wy = wy;
    out.wsv = wsv;
    out.edge = fabs((double)wsv - 40.0) < (double)kEdgeWsv || (grass && fabs((double)wsv - 1.0) < (double)kEdgeWsv);
    return out;
}

// FBP slope factor of a cell from its Horn numerators: SF = exp(3.533
// (GS/100)^1.2) with GS = 100 |g| / (8 cs) percent, capped at 10 from 70 %.
__device__ __forceinline__ double slope_factor(int gx, int gn, double cell_m) {
    if ((gx | gn) == 0) return 1.0;
    const double gs = 100.0 * sqrt((double)gx * (double)gx + (double)gn * (double)gn) / (8.0 * cell_m);
    return (gs >= 70.0) ? 10.0 : exp(3.533 * pow(gs / 100.0, 1.2));
}


// Lognormal rate multiplier with mean 1 for (cell, period, rep).
template <typename R>
__device__ __forceinline__ R noise_mult(uint64_t seed, uint32_t cell, uint32_t period, uint32_t rep,
                                        R sigma) {
    if (sigma == (R)0) return (R)1;
    const uint4 x = draw(seed, cell, period, rep, 0u);
    const R u1 = ((R)(x.x >> 8) + (R)1) * (R)(1.0 / 16777216.0);
    const R u2 = unit24<R>(x.y);
    const R z = m_sqrt((R)-2 * m_log(u1)) * cos_2pi(u2);
    return m_exp(sigma * z - (R)0.5 * sigma * sigma);
}

// Directional rates along the 8 axes (eq. (1)): with a = (H+B)/2 (eq. (2)),
// e^2 = 1 - 1/LB^2 (eq. (4) with FROS = a/LB), cos(phi) the cosine between
// the axis and the head direction, the front half (cos phi > 0) spreads at
// a(1-e^2)/(1 - e cos phi) and the back half at a(1-e^2).  Each rate is then
// scaled by the noise multiplier mu.  e is formed from LB - 1 directly and
// the denominator is evaluated as (1 - e) + e (1 - cos phi) with
// 1 - e = LB^-2 / (1 + e) and
// 1 - cos phi = |w/|w| - u|^2 / 2, which avoids the cancellation of
// 1 - e cos phi near the head direction when LB is large.
template <typename R>
__device__ __forceinline__ void axis_rates(const CellRates<R>& cr, R mu, R* x8) {
    const R a = (R)0.5 * (cr.h + cr.b);
    const R il = recip(cr.lb);
    const R il2 = il * il;
    const R base = a * il2;                           // a (1 - e^2)
    const R e = m_sqrt(cr.lbm1 * (cr.lbm1 + (R)2)) * il;   // sqrt(1 - 1/LB^2)
    const R one_m_e = il2 * recip((R)1 + e);
    const R inv_wsv = (cr.wsv > (R)0) ? recip(cr.wsv) : (R)0;
    const R cx = cr.wx * inv_wsv, cy = cr.wy * inv_wsv;   // unit head direction
    const R s = (R)0.70710678118654752440;
    const R ux[8] = {(R)1, s, (R)0, -s, (R)-1, -s, (R)0, s};
    const R uy[8] = {(R)0, s, (R)1, s, (R)0, -s, (R)-1, -s};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const R c = ux[k] * cx + uy[k] * cy;
        R r = base;
        if (c > (R)0) {
            const R dx = cx - ux[k], dy = cy - uy[k];
            r = base * recip(one_m_e + e * ((R)0.5 * (dx * dx + dy * dy)));
        }
        x8[k] = mu * r;
    }
}

// The same rates floored to integer m/min after adding u_k: 1/2, or the
// 24-bit uniforms of the words ua (axes 0-3) and ub (axes 4-7).
template <typename R>
__device__ __forceinline__ void axis_rates_q(const CellRates<R>& cr, R mu, bool stochastic, uint4 ua, uint4 ub,
                                             int32_t* q) {
    const R a = (R)0.5 * (cr.h + cr.b);
    const R il = recip(cr.lb);
    const R il2 = il * il;
    const R base = a * il2;
    const R e = m_sqrt(cr.lbm1 * (cr.lbm1 + (R)2)) * il;
    const R one_m_e = il2 * recip((R)1 + e);
    const R inv_wsv = (cr.wsv > (R)0) ? recip(cr.wsv) : (R)0;
    const R cx = cr.wx * inv_wsv, cy = cr.wy * inv_wsv;
    const R s = (R)0.70710678118654752440;
    const R ux[8] = {(R)1, s, (R)0, -s, (R)-1, -s, (R)0, s};
    const R uy[8] = {(R)0, s, (R)1, s, (R)0, -s, (R)-1, -s};
    const uint32_t w[8] = {ua.x, ua.y, ua.z, ua.w, ub.x, ub.y, ub.z, ub.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const R c = ux[k] * cx + uy[k] * cy;
        R r = base;
        if (c > (R)0) {
            const R dx = cx - ux[k], dy = cy - uy[k];
            r = base * recip(one_m_e + e * ((R)0.5 * (dx * dx + dy * dy)));
        }
        const R u = stochastic ? unit24<R>(w[k]) : (R)0.5;
        const R v = m_floor(mu * r + u);
        q[k] = (v < (R)1073741824) ? (int32_t)v : 1073741824;
    }
}

}  // namespace c2f

namespace c2f {

// FBP coefficient tables in each translation unit's constant memory.
static __constant__ CoefR<double> kCoef64[kNumFuels] = {C2F_FUEL_ROWS};
static __constant__ CoefR<float> kCoef32[kNumFuels] = {C2F_FUEL_ROWS};

template <typename R> __device__ __forceinline__ const CoefR<R>* coef_table();
template <> __device__ __forceinline__ const CoefR<double>* coef_table<double>() { return kCoef64; }
template <> __device__ __forceinline__ const CoefR<float>* coef_table<float>() { return kCoef32; }

template <typename R> __device__ __forceinline__ LandR<R> land_consts(const LandDev* L);
template <> __device__ __forceinline__ LandR<double> land_consts<double>(const LandDev* L) {
    return LandR<double>{L->pc_w64, L->cf64, L->cell_m64, L->pdf_w64, L->fme_r64, L->csi64};
}
template <> __device__ __forceinline__ LandR<float> land_consts<float>(const LandDev* L) {
    return LandR<float>{L->pc_w32, L->cf32, L->cell_m32, L->pdf_w32, L->fme_r32, L->csi32};
}

// Crown base height and crown fuel load per fuel.
static __constant__ CrownCoef kCrown[kNumFuels] = {C2F_CROWN_ROWS};

// Head fire intensity (kW/m) of a cell from its rates, before the noise
// multiplier: 300 TFC ROS with TFC = SFC + CFL CFB, the crown fraction
// burned CFB = 1 - exp(-0.23 (S - RSO)) above the critical surface rate RSO
// = CSI / (300 SFC) (S the head rate, the surface rate for C-6; 0 for fuels
// that do not crown).  *cfb (may be NULL) receives CFB.
template <typename R>
__device__ __forceinline__ R head_intensity(const CellRates<R>& cr, int f, const R* row, const LandR<R>& L,
                                            R* cfb_out) {
    R sfc = row[kRowSFC + f];
    if (is_mix_pc(f)) sfc = L.pc_w * row[kRowSFC + kC2] + ((R)1 - L.pc_w) * row[kRowSFC + kD1];
    const R cfl = (R)kCrown[f].cfl;
    R cfb = (R)0;
    if (cfl > (R)0 && sfc > (R)0) {
        const R rso = L.csi[f] * recip((R)300 * sfc);
        if (cr.rss > rso) cfb = -m_expm1((R)-0.23 * (cr.rss - rso));
    }
    if (cfb_out) *cfb_out = cfb;
    return (R)300 * (sfc + cfb * cfl) * cr.h;
}

// Everything a rate evaluation needs besides the cell: coefficient tables,
// landscape constants, the scenario's weather rows and the random stream.
template <typename R>
struct RateCtx {
    const CoefR<R>* coef;
    const CoefR<double>* coef64;
    LandR<R> L;
    LandR<double> L64;
    const R* rows;          // first row of the replication's scenario
    const double* rows64;
    // elements from one period's row to the next: kRowLen, or 0 where
    // rows, rows64 and rows32 hold only the period being evaluated
    uint32_t row_stride;
    uint64_t seed;
    R sigma;
    int rounding;
    uint32_t rep;
    float burnout;   // burn-out threshold on the integer axis rates (0 = off)
    float hfi_min;   // burn-out threshold on the head fire intensity, kW/m (0 = off)
    // FP32 coefficient table, landscape constants and weather rows of the
    // same scenario: an FP64 context tries them first (axis_q).  rows32
    // NULL: FP64 only.
    const CoefR<float>* coef32;
    LandR<float> L32;
    const float* rows32;
};

// Weather scenario and ignition cell of replication `rep` of a job
// (Section 3.1, uncertainty sources (1) and (3)): a fixed scenario or
// (x S) >> 32 from Philox tag 4; a fixed cell, the burnable cell (x |B|) >> 32
// of the row-major burnable list from tag 3, the burnable cell nearest the
// centre, or a draw from the ignition map: with running weight sums C and
// total W, the first cell whose C exceeds floor(x W / 2^32).  ign = -1 when
// there is nothing to ignite.
__device__ __forceinline__ void rep_draws(const Job& job, uint32_t rep, int& scen, int& ign) {
    scen = job.scen_fixed;
    if (job.scen_mode == 1) {
        const uint4 x = draw(job.seed, 0xFFFFFFFFu, 0xFFFFFFFFu, rep, 4u);
        scen = (int)(((uint64_t)x.x * (uint64_t)job.n_scen) >> 32);
    }
    ign = -1;
    if (job.ign_mode == 0) {
        ign = job.ign_cell;
    } else if (job.ign_mode == 1) {
        const int nbn = job.land->n_burnable;
        if (nbn > 0) {
            const uint4 x = draw(job.seed, 0xFFFFFFFFu, 0xFFFFFFFFu, rep, 3u);
            ign = job.burnable[((uint64_t)x.x * (uint64_t)nbn) >> 32];
        }
    } else if (job.ign_mode == 2) {
        ign = job.land->centre_cell;
    } else if (job.ign_mode == 4) {
        ign = job.n_seeds > 0 ? job.seeds[0].x : -1;   // the earliest entry of the list
    } else if (job.ign_total > 0) {
        const uint4 x = draw(job.seed, 0xFFFFFFFFu, 0xFFFFFFFFu, rep, 3u);
        const uint64_t W = job.ign_total;
        // floor(x W / 2^32) without overflow: W < 2^63
        const uint64_t t = (uint64_t)x.x * (W >> 32) + (((uint64_t)x.x * (W & 0xFFFFFFFFull)) >> 32);
        // first index with C[i] > t (C is non-decreasing, C[n-1] = W > t)
        int64_t lo = 0, hi = (int64_t)job.rows * job.cols - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (job.ign_cdf[mid] > t) hi = mid;
            else lo = mid + 1;
        }
        ign = (int)lo;
    }
}

// Does period p lie inside the daily burning window (the first burn_hours
// hours of every day from the start of the run; assumption A5)?  The
// period length divides 60 minutes whenever a window is set, so a period
// lies wholly inside or outside it.
__device__ __forceinline__ bool burning_period(const Job& job, int p) {
    if (job.burn_hours <= 0) return true;
    return (int)(((int64_t)p * job.period_min) % 1440) < job.burn_hours * 60;
}

// Does the ignition-point list hold an entry of period p?
__device__ __forceinline__ bool seeds_at(const Job& job, int p) {
    for (int k = 0; k < job.n_seeds; ++k)
        if (job.seeds[k].y == p) return true;
    return false;
}

// Integer axis rates (m/min) of a cell in a period: eq. (1) rates scaled by
// the noise multiplier, then floor(x + u) with u = 1/2 or a Philox uniform.
// Returns true when the cell burns out on its head fire intensity (A5 (iv)):
// an intensity threshold is set and the intensity, with the noise
// multiplier on the rate, is below it.
template <typename R>
__device__ __forceinline__ bool axis_q_direct(const RateCtx<R>& X, const CellRec& rec, uint32_t cell,
                                              uint32_t period, int32_t* q) {
    const size_t ro = (size_t)period * X.row_stride;
    const CellRates<R> cr = cell_rates<R>(X.coef, X.coef64, rec, X.rows + ro, X.rows64 + ro, X.L, X.L64);
    const R mu = noise_mult<R>(X.seed, cell, period, X.rep, X.sigma);
    uint4 ua = make_uint4(0u, 0u, 0u, 0u), ub = ua;
    if (X.rounding != 0) {
        ua = draw(X.seed, cell, period, X.rep, 1u);
        ub = draw(X.seed, cell, period, X.rep, 2u);
    }
    axis_rates_q<R>(cr, mu, X.rounding != 0, ua, ub, q);
    if (X.hfi_min > 0.f) {
        const R hfi = head_intensity<R>(cr, rec_fuel(rec.info), X.rows + ro, X.L, nullptr) * mu;
        return !((double)hfi >= (double)X.hfi_min);
    }
    return false;
}

// Integer rates of an FP64 context from an FP32 evaluation where that is
// exact.  Away from the speeds where the model's form jumps (f(W) at 40
// km/h, grass LB at 1 km/h), FP32 axis rates differ from the FP64 ones by
// at most 7.0e-6 of max(1, x) over 630 M rates of the 1024^2 batched
// landscape (its 16 fuel codes, 10 scenarios x 8 periods, noise, stochastic
// rounding) and 9.4e-6 over 5 harsh landscapes (all 18 fuels, slopes above
// 100 %, FFMC 80-99, BUI up to 250, winds up to 80 km/h), and head fire
// intensities by at most 4.5e-5 relative.  So where x32 + u lies more than
// kMixMargin max(1, x32) from an integer, floor(x64 + u) is the same
// integer, and where the FP32 intensity lies more than kMixMarginH of the
// threshold from it, the burn-out test agrees.  A cell whose FP32 wind
// speed lies within kEdgeWsv of a jump (CellRates::edge), and every lane
// where either test fails, takes the FP64 evaluation.  The margins leave a
// factor of three or more over the measured differences; every FP64 parity
// test compares the result with the FP64 oracle bit for bit.
constexpr double kMixMargin = 3e-5;
constexpr double kMixMarginH = 2e-4;

template <typename R>
__device__ __forceinline__ bool axis_q(const RateCtx<R>& X, const CellRec& rec, uint32_t cell, uint32_t period,
                                       int32_t* q) {
    if constexpr (sizeof(R) == 8) {
        if (X.rows32 != nullptr) {
            const size_t ro = (size_t)period * X.row_stride;
            const CellRates<float> cr =
                cell_rates<float>(X.coef32, X.coef64, rec, X.rows32 + ro, X.rows64 + ro, X.L32, X.L64);
            const float mu = noise_mult<float>(X.seed, cell, period, X.rep, (float)X.sigma);
            uint4 ua = make_uint4(0u, 0u, 0u, 0u), ub = ua;
            if (X.rounding != 0) {
                ua = draw(X.seed, cell, period, X.rep, 1u);
                ub = draw(X.seed, cell, period, X.rep, 2u);
            }
            float x[8];
            axis_rates<float>(cr, mu, x);
            const uint32_t w[8] = {ua.x, ua.y, ua.z, ua.w, ub.x, ub.y, ub.z, ub.w};
            bool exact = !cr.edge;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double u = X.rounding != 0 ? unit24<double>(w[k]) : 0.5;
                const double v = (double)x[k] + u;
                const double m = kMixMargin * fmax(1.0, (double)x[k]);
                const double lo = floor(v - m);
                exact = exact && lo == floor(v + m);
                q[k] = (lo < 1073741824.0) ? (int32_t)lo : 1073741824;
            }
            bool faint = false;
            if (X.hfi_min > 0.f) {
                const double hfi =
                    (double)(head_intensity<float>(cr, rec_fuel(rec.info), X.rows32 + ro, X.L32, nullptr) * mu);
                const double hm = (double)X.hfi_min;
                exact = exact && fabs(hfi - hm) > kMixMarginH * hm;
                faint = !(hfi >= hm);
            }
            if (exact) return faint;
        }
    }
    return axis_q_direct<R>(X, rec, cell, period, q);
}

// Head rate times the noise multiplier: the receiving cell's ignition test.
template <typename R>
__device__ __forceinline__ R head_rate(const RateCtx<R>& X, const CellRec& rec, uint32_t cell, uint32_t period) {
    const size_t ro = (size_t)period * X.row_stride;
    const CellRates<R> cr = cell_rates<R>(X.coef, X.coef64, rec, X.rows + ro, X.rows64 + ro, X.L, X.L64);
    return cr.h * noise_mult<R>(X.seed, cell, period, X.rep, X.sigma);
}

}  // namespace c2f
