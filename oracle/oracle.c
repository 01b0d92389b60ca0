/*
 * Cell2Fire reference oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain single-threaded C11, FP64 throughout, glibc libm.  It follows the
 * paper's steps in the paper's order:
 *   - cell model and 8-neighbour adjacency ....... Sections 3.1, 3.3, assumption A1
 *   - rate of spread per cell from the FBP System  Sections 2.3, 3.4 (step i), A2
 *   - ellipse fitting, eqs. (2)-(4) .............. Section 3.7
 *   - directional rate, eq. (1) (O'Regan 1976) ... Section 2.2
 *   - send/receive messages, one clock step at a
 *     time, synchronous update at step end ....... Section 3.1, Section 3.4 step ii,
 *                                                   Algorithm 1 Steps 0-3
 *   - burn-out when no neighbour is available .... assumption A5 (ii)
 *   - burn grids and probability counts .......... Section 3.6 (i)
 * The FBP System equations are not printed in the paper (it cites the
 * Forestry Canada 1992 ST-X-3 report); the forms used here are the public
 * FBP System ones, typed independently for this oracle.  The readings taken
 * where the paper is silent are listed at each function.
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846
#define D2R (PI / 180.0)

/* ---------------------------------------------------------------- Philox */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4]) {
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------ FBP System tables */
/* Fuel codes: 0 non-fuel, 1-7 C-1..C-7, 8 D-1, 9 M-1, 10 M-2, 11-13 S-1..S-3,
 * 14 O-1a, 15 O-1b, 16 D-2, 17 M-3, 18 M-4.  (Table FBPT shows the code ->
 * FBP type dictionary idea; the paper counts the FBP System's fuel types in
 * Section 2.3.) */
enum { NF = 0, C1 = 1, C2 = 2, C3 = 3, C4 = 4, C5 = 5, C6 = 6, C7 = 7, D1 = 8, M1 = 9, M2 = 10,
       S1 = 11, S2 = 12, S3 = 13, O1A = 14, O1B = 15, D2 = 16, M3 = 17, M4 = 18, NFUEL = 19 };

/* Rate-of-spread curve RSI = a (1 - exp(-b ISI))^c and BUI effect (q, BUI0).
 * M-3 and M-4 carry their dead-fir curves; M-1 and M-2 have none of their
 * own (they mix C-2 and D-1). */
static const double FBP_A[NFUEL] = {0, 90, 110, 110, 110, 30, 30, 45, 30, 0, 0, 75, 40, 55, 190, 250,
                                    6, 120, 100};
static const double FBP_B[NFUEL] = {0, 0.0649, 0.0282, 0.0444, 0.0293, 0.0697, 0.0800, 0.0305,
                                    0.0232, 0, 0, 0.0297, 0.0438, 0.0829, 0.0310, 0.0350,
                                    0.0232, 0.0572, 0.0404};
static const double FBP_C[NFUEL] = {0, 4.5, 1.5, 3.0, 1.5, 4.0, 3.0, 2.0, 1.6, 0, 0, 1.3, 1.7, 3.2, 1.4, 1.7,
                                    1.6, 1.4, 1.48};
static const double FBP_Q[NFUEL] = {0, 0.90, 0.70, 0.75, 0.80, 0.80, 0.80, 0.85, 0.90, 0.80, 0.80,
                                    0.75, 0.75, 0.75, 1.0, 1.0, 0.9, 0.8, 0.8};
static const double FBP_BUI0[NFUEL] = {0, 72, 64, 62, 66, 56, 62, 106, 32, 50, 50, 38, 63, 31, 1, 1,
                                       32, 50, 50};
/* Crown base height (m) and crown fuel load (kg/m^2) of the fuels that
 * crown (conifers and mixedwoods); 0 elsewhere. */
static const double FBP_CBH[NFUEL] = {0, 2, 3, 8, 4, 18, 7, 10, 0, 6, 6, 0, 0, 0, 0, 0, 0, 6, 6};
static const double FBP_CFL[NFUEL] = {0, 0.75, 0.8, 1.15, 1.2, 1.2, 1.8, 0.5, 0, 0.8, 0.8, 0, 0, 0, 0, 0,
                                      0, 0.8, 0.8};
#define GRASS_FUEL_LOAD 0.35 /* kg/m^2, O-1a and O-1b */

int oracle_fuel_coefficients(int32_t fuel, double* out5) {
    if (fuel < 1 || fuel >= NFUEL || !out5) return -1;
    out5[0] = FBP_A[fuel]; out5[1] = FBP_B[fuel]; out5[2] = FBP_C[fuel];
    out5[3] = FBP_Q[fuel]; out5[4] = FBP_BUI0[fuel];
    return 0;
}

int oracle_crown_coefficients(int32_t fuel, double* out2) {
    if (fuel < 1 || fuel >= NFUEL || !out2) return -1;
    out2[0] = FBP_CBH[fuel];
    out2[1] = FBP_CFL[fuel];
    return 0;
}

/* ------------------------------------------------------ FBP System model */

/* Landscape-wide FBP inputs: percent conifer (M-1/M-2), grass curing
 * (O-1), foliar moisture content (C-6 crown fire, crown fraction burned)
 * and percent dead fir (M-3/M-4), all in percent. */
typedef struct {
    double pc, cur, fmc, pdf;
} fbpland_t;

/* Fine fuel moisture content from FFMC, and the fine-fuel function f(F). */
static double fine_fuel_fn(double ffmc) {
    double m = 147.2 * (101.0 - ffmc) / (59.5 + ffmc);
    return 91.9 * exp(-0.1386 * m) * (1.0 + pow(m, 5.31) / 4.93e7);
}

/* Wind function f(W), W in km/h. */
static double wind_fn(double w) {
    if (w <= 40.0) return exp(0.05039 * w);
    return 12.0 * (1.0 - exp(-0.0818 * (w - 28.0)));
}

/* Rate of spread of a single (unmixed) fuel at initial spread index isi. */
static double rsi_pure(int f, double isi) {
    return FBP_A[f] * pow(-expm1(-FBP_B[f] * isi), FBP_C[f]);
}

/* Grass curing factor (percent curing c). */
static double curing_factor(double c) {
    if (c < 58.8) return 0.005 * (exp(0.061 * c) - 1.0);
    return 0.176 + 0.02 * (c - 58.8);
}

/* RSI for any fuel code.  M-1/M-2 mix C-2 and D-1 by percent conifer, M-3
 * /M-4 mix their dead-fir curve and D-1 by percent dead fir (M-2 and M-4
 * take 0.2 of the D-1 rate, the leaf-on stands); O-1 is scaled by the
 * curing factor; C-6 here is its surface curve (the crown part is added in
 * fbp_eval); D-2 has its own curve (a fifth of D-1's). */
static double rsi_fuel(int f, double isi, const fbpland_t* P) {
    double w = P->pc / 100.0, d = P->pdf / 100.0;
    switch (f) {
        case M1: return w * rsi_pure(C2, isi) + (1.0 - w) * rsi_pure(D1, isi);
        case M2: return w * rsi_pure(C2, isi) + 0.2 * (1.0 - w) * rsi_pure(D1, isi);
        case M3: return d * rsi_pure(M3, isi) + (1.0 - d) * rsi_pure(D1, isi);
        case M4: return d * rsi_pure(M4, isi) + 0.2 * (1.0 - d) * rsi_pure(D1, isi);
        case O1A:
        case O1B: return rsi_pure(f, isi) * curing_factor(P->cur);
        default: return rsi_pure(f, isi);
    }
}

/* Build-up effect; 1 when BUI is 0. */
static double bui_effect(int f, double bui) {
    if (bui <= 0.0) return 1.0;
    return exp(50.0 * log(FBP_Q[f]) * (1.0 / bui - 1.0 / FBP_BUI0[f]));
}

/* Inverse of the RSI curve: the spread index giving rate rsf (with the
 * 0.01 floor inside the logarithm); cf scales the curve's asymptote. */
static double isf_pure(int f, double rsf, double cf) {
    double t = 1.0 - pow(rsf / (cf * FBP_A[f]), 1.0 / FBP_C[f]);
    if (t < 0.01) t = 0.01;
    return log(t) / (-FBP_B[f]);
}

/* Slope-adjusted zero-wind spread index ISF.  Mixedwoods: the weighted ISF
 * of their two pure curves (percent conifer for M-1/M-2 over C-2 and D-1,
 * percent dead fir for M-3/M-4 over their own curve and D-1). */
static double isf_fuel(int f, double sf, double isz, const fbpland_t* P) {
    double w = P->pc / 100.0, d = P->pdf / 100.0;
    switch (f) {
        case M1:
        case M2:
            return w * isf_pure(C2, sf * rsi_pure(C2, isz), 1.0) +
                   (1.0 - w) * isf_pure(D1, sf * rsi_pure(D1, isz), 1.0);
        case M3:
        case M4:
            return d * isf_pure(f, sf * rsi_pure(f, isz), 1.0) +
                   (1.0 - d) * isf_pure(D1, sf * rsi_pure(D1, isz), 1.0);
        case O1A:
        case O1B: {
            double cf = curing_factor(P->cur);
            return isf_pure(f, sf * rsi_pure(f, isz) * cf, cf);
        }
        default: return isf_pure(f, sf * rsi_pure(f, isz), 1.0);
    }
}

/* Slope-equivalent wind speed WSE (km/h) for slope gs (percent). */
static double slope_equiv_wind(int f, double gs, double ff, const fbpland_t* P) {
    double sf = (gs >= 70.0) ? 10.0 : exp(3.533 * pow(gs / 100.0, 1.2));
    double isz = 0.208 * ff;
    double isf = isf_fuel(f, sf, isz, P);
    double wse = log(isf / isz) / 0.05039;
    if (wse > 40.0) {
        if (isf < 0.999 * 2.496 * ff) wse = 28.0 - log(1.0 - isf / (2.496 * ff)) / 0.0818;
        else wse = 112.45;
    }
    return wse;
}

/* Surface fuel consumption (kg/m^2) from FFMC and BUI. */
static double surface_fuel_consumption(int f, double ffmc, double bui, const fbpland_t* P) {
    switch (f) {
        case C1:
            return ffmc > 84.0 ? 0.75 + 0.75 * sqrt(1.0 - exp(-0.23 * (ffmc - 84.0)))
                               : 0.75 - 0.75 * sqrt(1.0 - exp(-0.23 * (84.0 - ffmc)));
        case C2:
        case M3:
        case M4: return 5.0 * (1.0 - exp(-0.0115 * bui));
        case C3:
        case C4: return 5.0 * pow(1.0 - exp(-0.0164 * bui), 2.24);
        case C5:
        case C6: return 5.0 * pow(1.0 - exp(-0.0149 * bui), 2.48);
        case C7: {
            double ffc = ffmc > 70.0 ? 2.0 * (1.0 - exp(-0.104 * (ffmc - 70.0))) : 0.0;
            return ffc + 1.5 * (1.0 - exp(-0.0201 * bui));
        }
        case D1:
        case D2: return 1.5 * (1.0 - exp(-0.0183 * bui));
        case M1:
        case M2: {
            double w = P->pc / 100.0;
            return w * 5.0 * (1.0 - exp(-0.0115 * bui)) + (1.0 - w) * 1.5 * (1.0 - exp(-0.0183 * bui));
        }
        case S1: return 4.0 * (1.0 - exp(-0.025 * bui)) + 4.0 * (1.0 - exp(-0.034 * bui));
        case S2: return 10.0 * (1.0 - exp(-0.013 * bui)) + 6.0 * (1.0 - exp(-0.060 * bui));
        case S3: return 12.0 * (1.0 - exp(-0.0166 * bui)) + 20.0 * (1.0 - exp(-0.0210 * bui));
        case O1A:
        case O1B: return GRASS_FUEL_LOAD;
        default: return 0.0;
    }
}

/* Critical surface fire intensity for crowning (kW/m) and the surface rate
 * it takes (m/min); the crown fraction burned at surface rate ros. */
static double critical_surface_rate(int f, double fmc, double sfc) {
    double csi = 0.001 * pow(FBP_CBH[f], 1.5) * pow(460.0 + 25.9 * fmc, 1.5);
    return sfc > 0.0 ? csi / (300.0 * sfc) : INFINITY;
}

static double crown_fraction(double ros, double rso) {
    return ros > rso ? 1.0 - exp(-0.23 * (ros - rso)) : 0.0;
}

/* C-6 crown fire rate at spread index isi: 60 (1 - exp(-0.0497 ISI)) scaled
 * by the foliar moisture effect relative to its average 0.778. */
static double c6_crown_rate(double isi, double fmc) {
    double fme = 1000.0 * pow(1.5 - 0.00275 * fmc, 4.0) / (460.0 + 25.9 * fmc);
    return 60.0 * (1.0 - exp(-0.0497 * isi)) * fme / 0.778;
}

typedef struct {
    double hros, bros, fros, lb, raz, isi, wsv, be, rsi, wse, sfc, cfb, tfc, hfi;
} fbp_t;

/* Head, back and flank rates, length-to-breadth ratio and spread azimuth,
 * and the head fire's fuel consumption and intensity.  Wind direction wd is
 * the azimuth the wind blows FROM; the fire heads downwind (wd + 180).  Slope
 * enters through the slope-equivalent wind, added as a vector along the
 * upslope azimuth saz.  C-6 adds its crown fire to the surface rate: ROS =
 * RSS + CFB (RSC - RSS) with CFB from the surface rate.  Crown fraction
 * burned, total fuel consumption SFC + CFB CFL and head fire intensity
 * 300 TFC ROS (kW/m) follow the head rate (the surface rate for C-6). */
static void fbp_eval(int f, double ffmc, double bui, double ws, double wd, double gs,
                     double saz, const fbpland_t* P, fbp_t* o) {
    double ff = fine_fuel_fn(ffmc);
    double wse = (gs > 0.0) ? slope_equiv_wind(f, gs, ff, P) : 0.0;
    double waz = fmod(wd + 180.0, 360.0);
    double wsx = ws * sin(waz * D2R) + wse * sin(saz * D2R);
    double wsy = ws * cos(waz * D2R) + wse * cos(saz * D2R);
    double wsv = sqrt(wsx * wsx + wsy * wsy);
    double raz = 0.0;
    if (wsv > 0.0) {
        double c = wsy / wsv;
        if (c > 1.0) c = 1.0;
        if (c < -1.0) c = -1.0;
        raz = acos(c) / D2R;
        if (wsx < 0.0) raz = 360.0 - raz;
    }
    double isi = 0.208 * wind_fn(wsv) * ff;
    double be = bui_effect(f, bui);
    double rsi = rsi_fuel(f, isi, P);
    double hros = rsi * be;
    double bisi = 0.208 * exp(-0.05039 * wsv) * ff;
    double bros = rsi_fuel(f, bisi, P) * be;
    double sfc = surface_fuel_consumption(f, ffmc, bui, P);
    double rso = critical_surface_rate(f, P->fmc, sfc);
    double cfb = 0.0;
    if (f == C6) {
        double rss = hros, brss = bros;
        cfb = crown_fraction(rss, rso);
        hros = rss + cfb * (c6_crown_rate(isi, P->fmc) - rss);
        bros = brss + crown_fraction(brss, rso) * (c6_crown_rate(bisi, P->fmc) - brss);
    } else if (FBP_CFL[f] > 0.0) {
        cfb = crown_fraction(hros, rso);
    }
    double lb;
    if (f == O1A || f == O1B) lb = (wsv >= 1.0) ? 1.1 * pow(wsv, 0.464) : 1.0;
    else lb = 1.0 + 8.729 * pow(1.0 - exp(-0.030 * wsv), 2.155);
    o->hros = hros;
    o->bros = bros;
    o->fros = (hros + bros) / (2.0 * lb); /* a = LB * b, Section 3.7 */
    o->lb = lb;
    o->raz = raz;
    o->isi = isi;
    o->wsv = wsv;
    o->be = be;
    o->rsi = rsi;
    o->wse = wse;
    o->sfc = sfc;
    o->cfb = cfb;
    o->tfc = sfc + cfb * FBP_CFL[f];
    o->hfi = 300.0 * o->tfc * hros;
}

int oracle_fbp_point_ext(int32_t fuel, double ffmc, double bui, double ws_kmh, double wd_from_deg,
                         double slope_pct, double upslope_az_deg, double pc_pct, double curing_pct,
                         double fmc_pct, double pdf_pct, double* out) {
    if (fuel < 1 || fuel >= NFUEL || !out) return -1;
    fbpland_t P = {pc_pct, curing_pct, fmc_pct, pdf_pct};
    fbp_t o;
    fbp_eval(fuel, ffmc, bui, ws_kmh, wd_from_deg, slope_pct, upslope_az_deg, &P, &o);
    out[0] = o.hros; out[1] = o.bros; out[2] = o.fros; out[3] = o.lb; out[4] = o.raz;
    out[5] = o.isi; out[6] = o.wsv; out[7] = o.be; out[8] = o.rsi; out[9] = o.wse;
    out[10] = o.sfc; out[11] = o.cfb; out[12] = o.tfc; out[13] = o.hfi;
    return 0;
}

int oracle_fbp_point(int32_t fuel, double ffmc, double bui, double ws_kmh, double wd_from_deg,
                     double slope_pct, double upslope_az_deg, double pc_pct, double curing_pct,
                     double* out) {
    double o[14];
    if (oracle_fbp_point_ext(fuel, ffmc, bui, ws_kmh, wd_from_deg, slope_pct, upslope_az_deg, pc_pct,
                             curing_pct, 97.0, 50.0, o))
        return -1;
    memcpy(out, o, 10 * sizeof(double));
    return 0;
}

/* ------------------------------------------- ellipse and eq. (1) per axis */

/* Axis k points at angle theta_k = 45 k degrees (0 = East, counter-clockwise,
 * Section 3.4 step i): E, NE, N, NW, W, SW, S, SE. */
static const int AX_DR[8] = {0, -1, -1, -1, 0, 1, 1, 1};
static const int AX_DC[8] = {1, 1, 0, -1, -1, -1, 0, 1};

void oracle_axis_ros(double hros, double bros, double fros, double raz_deg, double* out8) {
    /* eq. (2) with t = 1: semi-major axis rate; eq. (4): eccentricity. */
    double a = (hros + bros) / 2.0;
    double e = 0.0;
    if (a > 0.0) {
        double r = fros / a;
        double s = 1.0 - r * r;
        e = (s > 0.0) ? sqrt(s) : 0.0;
    }
    double theta_head = 90.0 - raz_deg; /* azimuth -> counter-clockwise from East */
    for (int k = 0; k < 8; ++k) {
        double phi = 45.0 * k - theta_head;
        double c = cos(phi * D2R);
        /* eq. (1): front half uses the focal polar form, back half a(1-e^2). */
        out8[k] = (c > 0.0) ? a * (1.0 - e * e) / (1.0 - e * c) : a * (1.0 - e * e);
    }
}

/* ------------------------------------------------------------ landscape */

typedef struct {
    int32_t rows, cols, cell_m;
    const uint8_t* fuel;
    const int16_t* elev;
    fbpland_t P;
    int32_t n_scen, n_wp;
    const float* weather;
    int32_t d[8]; /* centre-to-centre distance per axis, integer metres */
} land_t;

static int16_t elev_at(const land_t* L, int r, int c) {
    if (r < 0) r = 0;
    if (r >= L->rows) r = L->rows - 1;
    if (c < 0) c = 0;
    if (c >= L->cols) c = L->cols - 1;
    return L->elev ? L->elev[(size_t)r * L->cols + c] : 0;
}

/* Horn's 3x3 finite-difference gradient (integer numerators). */
static void horn(const land_t* L, int r, int c, int32_t* gx, int32_t* gn) {
#define Z(dr, dc) ((int32_t)elev_at(L, r + (dr), c + (dc)))
    *gx = (Z(-1, 1) + 2 * Z(0, 1) + Z(1, 1)) - (Z(-1, -1) + 2 * Z(0, -1) + Z(1, -1));
    *gn = (Z(-1, -1) + 2 * Z(-1, 0) + Z(-1, 1)) - (Z(1, -1) + 2 * Z(1, 0) + Z(1, 1));
#undef Z
}

int oracle_horn(int32_t rows, int32_t cols, const int16_t* elev, int32_t* gx, int32_t* gn) {
    if (rows <= 0 || cols <= 0 || !gx || !gn) return -1;
    land_t L;
    memset(&L, 0, sizeof L);
    L.rows = rows; L.cols = cols; L.elev = elev;
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c) horn(&L, r, c, &gx[(size_t)r * cols + c], &gn[(size_t)r * cols + c]);
    return 0;
}

/* Slope (percent) and upslope azimuth (degrees clockwise from north). */
static void cell_slope(const land_t* L, int cell, double* gs, double* saz) {
    int32_t gx, gn;
    horn(L, cell / L->cols, cell % L->cols, &gx, &gn);
    double g = sqrt((double)gx * gx + (double)gn * gn);
    *gs = 100.0 * g / (8.0 * L->cell_m);
    *saz = (g > 0.0) ? fmod(atan2((double)gx, (double)gn) / D2R + 360.0, 360.0) : 0.0;
}

static int neighbour(const land_t* L, int cell, int k) {
    int r = cell / L->cols + AX_DR[k];
    int c = cell % L->cols + AX_DC[k];
    if (r < 0 || r >= L->rows || c < 0 || c >= L->cols) return -1;
    return r * L->cols + c;
}

/* ------------------------------------------------ per (cell, period) rates */

typedef struct {
    double h, b, f, lb, raz, mu, cfb, hfi;
    double x[8], xu[8];
    int32_t q[8];
} cellros_t;

/* Lognormal multiplier with mean 1: exp(sigma Z - sigma^2/2), Z by Box-Muller. */
static double noise_mu(uint64_t seed, int cell, int period, int rep, double sigma) {
    if (sigma == 0.0) return 1.0;
    uint32_t x[4];
    draw(seed, (uint32_t)cell, (uint32_t)period, (uint32_t)rep, 0u, x);
    double u1 = ((double)(x[0] >> 8) + 1.0) * (1.0 / 16777216.0);
    double u2 = (double)(x[1] >> 8) * (1.0 / 16777216.0);
    double z = sqrt(-2.0 * log(u1)) * cos(2.0 * PI * u2);
    return exp(sigma * z - 0.5 * sigma * sigma);
}

static void cell_fbp(const land_t* L, int cell, int scen, int period, fbp_t* o) {
    const float* w = L->weather + ((size_t)scen * L->n_wp + period) * 4;
    double gs, saz;
    cell_slope(L, cell, &gs, &saz);
    fbp_eval(L->fuel[cell], (double)w[0], (double)w[1], (double)w[2], (double)w[3], gs, saz, &L->P, o);
}

static void cell_ros(const land_t* L, int cell, int scen, int period, int rep, uint64_t seed,
                     double sigma, int rounding, cellros_t* out) {
    fbp_t o;
    cell_fbp(L, cell, scen, period, &o);
    double mu = noise_mu(seed, cell, period, rep, sigma);
    double ros[8];
    oracle_axis_ros(o.hros, o.bros, o.fros, o.raz, ros);
    double u[8];
    if (rounding == 0) {
        for (int k = 0; k < 8; ++k) u[k] = 0.5;
    } else {
        uint32_t a[4], b[4];
        draw(seed, (uint32_t)cell, (uint32_t)period, (uint32_t)rep, 1u, a);
        draw(seed, (uint32_t)cell, (uint32_t)period, (uint32_t)rep, 2u, b);
        for (int k = 0; k < 4; ++k) {
            u[k] = (double)(a[k] >> 8) * (1.0 / 16777216.0);
            u[k + 4] = (double)(b[k] >> 8) * (1.0 / 16777216.0);
        }
    }
    out->h = o.hros * mu;
    out->b = o.bros * mu;
    out->f = o.fros * mu;
    out->lb = o.lb;
    out->raz = o.raz;
    out->mu = mu;
    /* the multiplier scales the spread rate; the fuel consumed (and so the
     * crown fraction burned) is the FBP System's own */
    out->cfb = o.cfb;
    out->hfi = o.hfi * mu;
    for (int k = 0; k < 8; ++k) {
        out->x[k] = mu * ros[k];
        out->xu[k] = out->x[k] + u[k];
        out->q[k] = (int32_t)floor(out->xu[k]);
    }
}

/* ------------------------------------------------------------ validation */

static int check_land(int32_t rows, int32_t cols, int32_t cell_m, const uint8_t* fuel,
                      const fbpland_t* P, int32_t n_scen, int32_t n_wp, const float* weather) {
    if (rows <= 0 || cols <= 0 || cell_m <= 0 || cell_m > 20000 || !fuel || !weather) return -1;
    if ((int64_t)rows * cols > 0x7FFFFFFEll) return -1;
    if (!(P->pc >= 0.0 && P->pc <= 100.0) || !(P->cur > 0.0 && P->cur <= 100.0)) return -1;
    if (!(P->fmc > 0.0 && P->fmc <= 300.0) || !(P->pdf >= 0.0 && P->pdf <= 100.0)) return -1;
    if (n_scen <= 0 || n_wp <= 0) return -1;
    for (int64_t i = 0; i < (int64_t)rows * cols; ++i)
        if (fuel[i] >= NFUEL) return -1;
    for (int64_t i = 0; i < (int64_t)n_scen * n_wp; ++i) {
        const float* w = weather + i * 4;
        if (!(w[0] >= 0.0f && w[0] <= 101.0f) || !(w[1] >= 0.0f) || !(w[2] >= 0.0f) ||
            !isfinite(w[1]) || !isfinite(w[2]) || !isfinite(w[3]))
            return -1;
    }
    return 0;
}

static void init_land(land_t* L, int32_t rows, int32_t cols, int32_t cell_m, const uint8_t* fuel,
                      const int16_t* elev, const fbpland_t* P, int32_t n_scen, int32_t n_wp,
                      const float* weather) {
    L->rows = rows; L->cols = cols; L->cell_m = cell_m; L->fuel = fuel; L->elev = elev;
    L->P = *P; L->n_scen = n_scen; L->n_wp = n_wp; L->weather = weather;
    /* Orthogonal neighbours sit one cell width away; diagonal ones sqrt(2)
     * widths, rounded up to whole metres (least D with D*D >= 2 cs^2). */
    int64_t two = 2ll * cell_m * cell_m;
    int64_t dd = (int64_t)sqrt((double)two);
    while (dd * dd < two) ++dd;
    while ((dd - 1) * (dd - 1) >= two) --dd;
    for (int k = 0; k < 8; ++k) L->d[k] = (k % 2 == 0) ? cell_m : (int32_t)dd;
}

int oracle_eval_ros(int32_t rows, int32_t cols, int32_t cell_m, const uint8_t* fuel,
                    const int16_t* elev, double pc_pct, double curing_pct,
                    int32_t n_scen, int32_t n_wperiods, const float* weather,
                    int32_t scenario, int32_t period, int32_t rep, uint64_t seed, double sigma,
                    int32_t rounding, double* hros, double* bros, double* fros, double* lb,
                    double* raz, double* x8, double* xu8, int32_t* q8) {
    return oracle_eval_ros_cells(rows, cols, cell_m, fuel, elev, pc_pct, curing_pct, 97.0, 50.0, n_scen,
                                 n_wperiods, weather, scenario, period, rep, seed, sigma, rounding, -1, NULL,
                                 hros, bros, fros, lb, raz, x8, xu8, q8, NULL, NULL);
}

int oracle_eval_ros_cells(int32_t rows, int32_t cols, int32_t cell_m, const uint8_t* fuel,
                          const int16_t* elev, double pc_pct, double curing_pct, double fmc_pct,
                          double pdf_pct, int32_t n_scen, int32_t n_wperiods, const float* weather,
                          int32_t scenario, int32_t period, int32_t rep, uint64_t seed, double sigma,
                          int32_t rounding, int64_t n_cells, const int32_t* cells, double* hros,
                          double* bros, double* fros, double* lb, double* raz, double* x8, double* xu8,
                          int32_t* q8, double* cfb, double* hfi) {
    const fbpland_t P = {pc_pct, curing_pct, fmc_pct, pdf_pct};
    if (check_land(rows, cols, cell_m, fuel, &P, n_scen, n_wperiods, weather)) return -1;
    if (scenario < 0 || scenario >= n_scen || period < 0 || period >= n_wperiods || rep < 0) return -1;
    if (!(sigma >= 0.0) || (rounding != 0 && rounding != 1)) return -1;
    land_t L;
    init_land(&L, rows, cols, cell_m, fuel, elev, &P, n_scen, n_wperiods, weather);
    const int64_t n = cells ? n_cells : (int64_t)rows * cols;
    for (int64_t k = 0; k < n; ++k) {
        if (cells && (cells[k] < 0 || (int64_t)cells[k] >= (int64_t)rows * cols)) return -1;
    }
    for (int64_t o = 0; o < n; ++o) {
        const int64_t i = cells ? cells[o] : o;   /* grid cell; outputs are indexed by o */
        cellros_t c;
        if (fuel[i] == 0) {
            memset(&c, 0, sizeof c);
        } else {
            cell_ros(&L, (int)i, scenario, period, rep, seed, sigma, rounding, &c);
        }
        if (hros) hros[o] = c.h;
        if (bros) bros[o] = c.b;
        if (fros) fros[o] = c.f;
        if (lb) lb[o] = c.lb;
        if (raz) raz[o] = c.raz;
        if (cfb) cfb[o] = c.cfb;
        if (hfi) hfi[o] = c.hfi;
        for (int k = 0; k < 8; ++k) {
            if (x8) x8[o * 8 + k] = c.x[k];
            if (xu8) xu8[o * 8 + k] = c.xu[k];
            if (q8) q8[o * 8 + k] = c.q[k];
        }
    }
    return 0;
}

/* ------------------------------------------------------------ simulation */

typedef struct {
    int32_t cell;
    int32_t qperiod;
    int32_t q[8];
    int64_t prog[8]; /* metres travelled along each axis */
} burning_t;

typedef struct {
    int32_t n;
    const int32_t* key; /* sorted (rep, period, cell) */
    const int32_t* q;
} override_t;

static int key_cmp(const int32_t* a, const int32_t* b) {
    for (int i = 0; i < 3; ++i) {
        if (a[i] < b[i]) return -1;
        if (a[i] > b[i]) return 1;
    }
    return 0;
}

static const int32_t* override_find(const override_t* ov, int rep, int period, int cell) {
    int32_t k[3] = {rep, period, cell};
    int lo = 0, hi = ov->n - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        int c = key_cmp(ov->key + 3 * mid, k);
        if (c == 0) return ov->q + 8 * mid;
        if (c < 0) lo = mid + 1;
        else hi = mid - 1;
    }
    return NULL;
}

#define INF_T INT32_MAX

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
                    int32_t* scenario_out, int64_t* stats) {
    return oracle_simulate_ext(rows, cols, cell_m, fuel, elev, pc_pct, curing_pct, 97.0, 50.0, n_scen,
                               n_wperiods, period_min, weather, reps, rep_offset, n_periods, seed, sigma,
                               threshold, rounding, ignition_mode, ignition_cell, NULL, 0, 0, 0.0, 0.0, 0, NULL,
                               scenario_mode, scenario_fixed, n_override, override_key, override_q, scar, arrival_period,
                               arrival_minute, burn_count, burned_cells, ignition_out, scenario_out, stats);
}

/* Is minute m (1-based) inside the daily burning window: the first
 * burn_hours hours of every 24 h counted from the start of the run
 * (assumption A5, general fire dynamics (1)); burn_hours 0 = every minute. */
static int burning_minute(int32_t m, int32_t burn_hours) {
    if (burn_hours <= 0) return 1;
    return ((m - 1) % 1440) < burn_hours * 60;
}

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
                        int32_t* scenario_out, int64_t* stats) {
    if (!(burnout_ros >= 0.0) || !isfinite(burnout_ros)) return -1;
    if (!(hfi_min >= 0.0) || !isfinite(hfi_min)) return -1;
    const fbpland_t FP = {pc_pct, curing_pct, fmc_pct, pdf_pct};
    if (check_land(rows, cols, cell_m, fuel, &FP, n_scen, n_wperiods, weather)) return -1;
    if (reps <= 0 || rep_offset < 0 || n_periods <= 0 || n_periods > n_wperiods || period_min <= 0)
        return -1;
    if ((int64_t)n_periods * period_min > 0x7FFFFFF0ll) return -1;
    if (!(sigma >= 0.0) || !isfinite(threshold) || (rounding != 0 && rounding != 1)) return -1;
    const int64_t n = (int64_t)rows * cols;
    if (ignition_mode < 0 || ignition_mode > 4) return -1;
    if (ignition_mode == 0 && (ignition_cell < 0 || ignition_cell >= n)) return -1;
    if (ignition_mode == 3 && !ignition_weights) return -1;
    if (ignition_period < 0 || ignition_period >= n_periods) return -1;
    if (ignition_mode == 4) {
        if (n_ignitions < 1 || !ignition_list) return -1;
        for (int32_t k = 0; k < n_ignitions; ++k) {
            const int32_t c = ignition_list[2 * k], p = ignition_list[2 * k + 1];
            if (c < 0 || c >= n || p < 0 || p >= n_periods) return -1;
        }
    }
    if (burn_hours < 0 || burn_hours > 24) return -1;
    if (scenario_mode < 0 || scenario_mode > 1) return -1;
    if (scenario_mode == 0 && (scenario_fixed < 0 || scenario_fixed >= n_scen)) return -1;
    if (n_override < 0 || (n_override > 0 && (!override_key || !override_q))) return -1;

    land_t L;
    init_land(&L, rows, cols, cell_m, fuel, elev, &FP, n_scen, n_wperiods, weather);
    const int32_t P = period_min;
    const int32_t T = n_periods * period_min;

    /* q overrides, sorted by key for lookup */
    override_t ov = {0, NULL, NULL};
    int32_t* ov_key = NULL;
    int32_t* ov_q = NULL;
    if (n_override > 0) {
        ov_key = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)n_override);
        ov_q = (int32_t*)malloc(sizeof(int32_t) * 8 * (size_t)n_override);
        int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_override);
        for (int i = 0; i < n_override; ++i) order[i] = i;
        /* insertion sort: override lists are short */
        for (int i = 1; i < n_override; ++i) {
            int32_t v = order[i];
            int j = i - 1;
            while (j >= 0 && key_cmp(override_key + 3 * order[j], override_key + 3 * v) > 0) {
                order[j + 1] = order[j];
                --j;
            }
            order[j + 1] = v;
        }
        for (int i = 0; i < n_override; ++i) {
            memcpy(ov_key + 3 * i, override_key + 3 * order[i], 3 * sizeof(int32_t));
            memcpy(ov_q + 8 * i, override_q + 8 * order[i], 8 * sizeof(int32_t));
        }
        free(order);
        ov.n = n_override; ov.key = ov_key; ov.q = ov_q;
    }

    /* burnable cells in row-major order (uniform ignition) */
    int64_t n_burnable = 0;
    for (int64_t i = 0; i < n; ++i) n_burnable += (fuel[i] != 0);
    int32_t* burnable = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_burnable > 0 ? n_burnable : 1));
    {
        int64_t k = 0;
        for (int64_t i = 0; i < n; ++i)
            if (fuel[i] != 0) burnable[k++] = (int32_t)i;
    }
    /* burnable cell nearest to the centre (rows/2, cols/2) */
    int32_t centre_cell = -1;
    {
        int64_t best = INT64_MAX;
        int cr = rows / 2, cc = cols / 2;
        for (int64_t i = 0; i < n; ++i) {
            if (fuel[i] == 0) continue;
            int64_t dr = i / cols - cr, dc = i % cols - cc;
            int64_t d = dr * dr + dc * dc;
            if (d < best) { best = d; centre_cell = (int32_t)i; }
        }
    }

    /* ignition-point list (Section 3.2 (iii): cells paired with their
     * ignition periods), ordered by period; entries of one period keep the
     * given order (insertion sort, stable) */
    int32_t n_seed = ignition_mode == 4 ? n_ignitions : 0;
    int32_t* seeds = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(n_seed > 0 ? n_seed : 1));
    for (int32_t i = 0; i < n_seed; ++i) {
        int32_t c = ignition_list[2 * i], p = ignition_list[2 * i + 1];
        int32_t j = i - 1;
        while (j >= 0 && seeds[2 * j + 1] > p) {
            seeds[2 * (j + 1)] = seeds[2 * j];
            seeds[2 * (j + 1) + 1] = seeds[2 * j + 1];
            --j;
        }
        seeds[2 * (j + 1)] = c;
        seeds[2 * (j + 1) + 1] = p;
    }

    /* total ignition weight (spatial ignition map) */
    uint64_t ign_total = 0;
    if (ignition_mode == 3)
        for (int64_t i = 0; i < n; ++i) ign_total += ignition_weights[i];

    int32_t* arrival = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t* reached = (uint8_t*)malloc((size_t)n);
    int32_t* pending = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    size_t cap = 1024;
    burning_t* burn = (burning_t*)malloc(sizeof(burning_t) * cap);
    if (burn_count) memset(burn_count, 0, sizeof(uint32_t) * (size_t)n);
    int64_t st_ign = 0, st_bcm = 0, st_fbp = 0, st_bp = 0, st_ax = 0;

    for (int32_t lr = 0; lr < reps; ++lr) {
        const int32_t rep = rep_offset + lr;
        uint32_t x[4];
        /* Step 0 / Step 1 of Algorithm 1: scenario and ignition choice */
        int32_t scen = scenario_fixed;
        if (scenario_mode == 1) {
            draw(seed, 0xFFFFFFFFu, 0xFFFFFFFFu, (uint32_t)rep, 4u, x);
            scen = (int32_t)(((uint64_t)x[0] * (uint64_t)n_scen) >> 32);
        }
        int32_t ign = -1;
        if (ignition_mode == 0) {
            ign = ignition_cell;
        } else if (ignition_mode == 1) {
            if (n_burnable > 0) {
                draw(seed, 0xFFFFFFFFu, 0xFFFFFFFFu, (uint32_t)rep, 3u, x);
                ign = burnable[((uint64_t)x[0] * (uint64_t)n_burnable) >> 32];
            }
        } else if (ignition_mode == 2) {
            ign = centre_cell;
        } else if (ignition_mode == 4) {
            ign = seeds[0];
        } else {
            /* spatial ignition probability (Section 3.1, uncertainty (1)):
             * cell i with probability w_i / W.  The draw x (32 bits, tag 3)
             * picks the target t = floor(x W / 2^32) in [0, W) and the
             * ignition is the first cell whose running weight sum exceeds t. */
            if (ign_total > 0) {
                draw(seed, 0xFFFFFFFFu, 0xFFFFFFFFu, (uint32_t)rep, 3u, x);
                const uint64_t t = (uint64_t)x[0] * (ign_total >> 32) +
                                   (((uint64_t)x[0] * (ign_total & 0xFFFFFFFFull)) >> 32);
                uint64_t run = 0;
                for (int64_t i = 0; i < n; ++i) {
                    run += ignition_weights[i];
                    if (run > t) {
                        ign = (int32_t)i;
                        break;
                    }
                }
            }
        }
        for (int64_t i = 0; i < n; ++i) arrival[i] = INF_T;
        memset(reached, 0, (size_t)n);
        size_t nb = 0, np = 0;
        /* the ignition takes the last minute before its period; a list's
         * fires are lit as the clock reaches their periods (below) */
        const int32_t m0 = (ignition_mode == 4 ? seeds[1] : ignition_period) * P;
        int32_t si = 0;   /* next list entry to light */
        if (ignition_mode != 4 && ign >= 0 && fuel[ign] != 0) {
            arrival[ign] = m0;
            burn[0].cell = ign;
            burn[0].qperiod = -1;
            for (int k = 0; k < 8; ++k) burn[0].prog[k] = 0;
            nb = 1;
            ++st_ign;
        }
        /* Step 2: fire dynamics, one clock minute at a time; outside the
         * daily burning window nothing spreads or ignites */
        for (int32_t m = m0 + 1; m <= T && (nb > 0 || np > 0 || si < n_seed); ++m) {
            /* list ignitions of period p take minute p P: lit before minute
             * p P + 1 is stepped, inside or outside the burning window, on a
             * cell with fuel that has not burned yet (a reached cell waiting
             * on the threshold included) */
            while (si < n_seed && seeds[2 * si + 1] * P <= m - 1) {
                const int32_t c = seeds[2 * si];
                if (fuel[c] != 0 && arrival[c] == INF_T) {
                    arrival[c] = seeds[2 * si + 1] * P;
                    if (nb == cap) {
                        cap *= 2;
                        burn = (burning_t*)realloc(burn, sizeof(burning_t) * cap);
                    }
                    burn[nb].cell = c;
                    burn[nb].qperiod = -1;
                    for (int k = 0; k < 8; ++k) burn[nb].prog[k] = 0;
                    ++nb;
                    ++st_ign;
                }
                ++si;
            }
            if (!burning_minute(m, burn_hours)) continue;
            const int32_t p = (m - 1) / P;
            /* sending: every burning cell advances its fire along each axis
             * towards an available neighbour; reaching the neighbour's centre
             * sends it a message */
            for (size_t bi = 0; bi < nb; ++bi) {
                burning_t* b = &burn[bi];
                if (b->qperiod != p) {
                    /* a burning-cell-period: the cell's rates for p are taken
                     * while some axis still leads to an available neighbour */
                    for (int k = 0; k < 8; ++k) {
                        int j = neighbour(&L, b->cell, k);
                        if (j >= 0 && fuel[j] != 0 && arrival[j] == INF_T && b->prog[k] < L.d[k]) {
                            ++st_bp;
                            break;
                        }
                    }
                    const int32_t* oq = ov.n ? override_find(&ov, rep, p, b->cell) : NULL;
                    cellros_t c;
                    if (!oq || hfi_min > 0.0) {
                        cell_ros(&L, b->cell, scen, p, rep, seed, sigma, rounding, &c);
                        ++st_fbp;
                    }
                    for (int k = 0; k < 8; ++k) b->q[k] = oq ? oq[k] : c.q[k];
                    b->qperiod = p;
                    /* burn-out (A5 iv): a head fire intensity below the
                     * user's threshold makes the cell unavailable */
                    if (hfi_min > 0.0 && c.hfi < hfi_min)
                        for (int k = 0; k < 8; ++k) b->prog[k] = L.d[k];
                    /* burn-out (A5 i): when the rates toward every burnable
                     * neighbour fall below delta the cell stops spreading */
                    if (burnout_ros > 0.0) {
                        int32_t qmax = 0;
                        for (int k = 0; k < 8; ++k) {
                            int j = neighbour(&L, b->cell, k);
                            if (j >= 0 && fuel[j] != 0 && b->q[k] > qmax) qmax = b->q[k];
                        }
                        if ((double)qmax < burnout_ros)
                            for (int k = 0; k < 8; ++k) b->prog[k] = L.d[k];
                    }
                }
                for (int k = 0; k < 8; ++k) {
                    int j = neighbour(&L, b->cell, k);
                    if (j < 0 || fuel[j] == 0 || arrival[j] != INF_T || b->prog[k] >= L.d[k]) continue;
                    b->prog[k] += b->q[k];
                    if (b->prog[k] >= L.d[k]) {
                        ++st_ax;   /* an axis reach event: the neighbour's centre is reached */
                        b->prog[k] = L.d[k];
                        if (!reached[j]) {
                            reached[j] = 1;
                            pending[np++] = j;
                        }
                    }
                }
            }
            st_bcm += (int64_t)nb;
            /* receiving (synchronous, end of step): a reached cell ignites
             * if its own rate of spread exceeds the threshold now; otherwise
             * it stays reached and is re-examined at later steps */
            size_t keep = 0;
            for (size_t pi = 0; pi < np; ++pi) {
                int j = pending[pi];
                if (arrival[j] != INF_T) continue;
                int ok;
                if (threshold < 0.0) {
                    ok = 1;
                } else {
                    fbp_t o;
                    cell_fbp(&L, j, scen, p, &o);
                    ++st_fbp;
                    ok = (o.hros * noise_mu(seed, j, p, rep, sigma) > threshold);
                }
                if (ok) {
                    arrival[j] = m;
                    if (nb == cap) {
                        cap *= 2;
                        burn = (burning_t*)realloc(burn, sizeof(burning_t) * cap);
                    }
                    burn[nb].cell = j;
                    burn[nb].qperiod = -1;
                    for (int k = 0; k < 8; ++k) burn[nb].prog[k] = 0;
                    ++nb;
                    ++st_ign;
                } else {
                    pending[keep++] = j;
                }
            }
            np = keep;
            /* burn-out (A5 ii): drop cells with no axis left to an available neighbour */
            size_t w = 0;
            for (size_t bi = 0; bi < nb; ++bi) {
                burning_t* b = &burn[bi];
                int live = 0;
                for (int k = 0; k < 8 && !live; ++k) {
                    int j = neighbour(&L, b->cell, k);
                    if (j >= 0 && fuel[j] != 0 && arrival[j] == INF_T && b->prog[k] < L.d[k]) live = 1;
                }
                if (live) burn[w++] = *b;
            }
            nb = w;
        }
        /* Step 3: outputs */
        int64_t burned = 0;
        for (int64_t i = 0; i < n; ++i) {
            int32_t a = arrival[i];
            int on = (a != INF_T);
            burned += on;
            size_t o = (size_t)lr * (size_t)n + (size_t)i;
            if (scar) scar[o] = (uint8_t)on;
            if (arrival_minute) arrival_minute[o] = on ? a : -1;
            if (arrival_period) arrival_period[o] = !on ? -1 : (a == 0 ? 0 : (a - 1) / P);
            if (burn_count && on) burn_count[i] += 1u;
        }
        if (burned_cells) burned_cells[lr] = burned;
        if (ignition_out) ignition_out[lr] = ign;
        if (scenario_out) scenario_out[lr] = scen;
    }
    if (stats) {
        stats[0] = st_ign;
        stats[1] = st_bcm;
        stats[2] = st_fbp;
        stats[3] = st_bp;
        stats[4] = st_ax;
    }
    free(seeds);
    free(burn);
    free(pending);
    free(reached);
    free(arrival);
    free(burnable);
    free(ov_key);
    free(ov_q);
    return 0;
}

/* Scar comparison of Section 4 (comparison methodology): for t = 1..T the
 * simulated scar Y^t (cells whose arrival minute is in [0, t P]) against the
 * reference 0-1 scar X^t = reference[t-1][.], by mean squared error and the
 * structural similarity of Wang et al. (2004), evaluated over the whole grid
 * with C1 = (0.01 L)^2, C2 = (0.03 L)^2, L = 1, standard deviations and
 * covariance normalised by N - 1, and the denominator (mu_x^2 + mu_y^2 + C1)
 * (sigma_x^2 + sigma_y^2 + C2) (the printed formula repeats the means in the
 * second factor); delta_norm is the Frobenius norm of X^T - Y^T. */
int oracle_scar_metrics(int64_t n_cells, int32_t n_periods, int32_t period_min, const int32_t* arrival_minute,
                        const uint8_t* reference, double* mse, double* ssim, double* delta_norm) {
    if (n_cells < 2 || n_periods < 1 || period_min < 1 || !arrival_minute || !reference) return -1;
    const double N = (double)n_cells;
    const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
    for (int32_t t = 1; t <= n_periods; ++t) {
        const uint8_t* X = reference + (size_t)(t - 1) * (size_t)n_cells;
        const int64_t end = (int64_t)t * period_min;
        double sx = 0.0, sy = 0.0;
        for (int64_t i = 0; i < n_cells; ++i) {
            sx += (double)(X[i] != 0);
            sy += (double)(arrival_minute[i] >= 0 && arrival_minute[i] <= end);
        }
        const double mx = sx / N, my = sy / N;
        double vx = 0.0, vy = 0.0, cxy = 0.0, se = 0.0;
        for (int64_t i = 0; i < n_cells; ++i) {
            const double x = (double)(X[i] != 0);
            const double y = (double)(arrival_minute[i] >= 0 && arrival_minute[i] <= end);
            vx += (x - mx) * (x - mx);
            vy += (y - my) * (y - my);
            cxy += (x - mx) * (y - my);
            se += (x - y) * (x - y);
        }
        vx /= (N - 1.0);
        vy /= (N - 1.0);
        cxy /= (N - 1.0);
        if (mse) mse[t - 1] = se / N;
        if (ssim) ssim[t - 1] = ((2.0 * mx * my + C1) * (2.0 * cxy + C2)) / ((mx * mx + my * my + C1) * (vx + vy + C2));
        if (delta_norm && t == n_periods) *delta_norm = sqrt(se);
    }
    return 0;
}
