// FBP System fuel coefficients used by the device code and reported by
// c2f_fbp_coefficients().  Rate-of-spread curve RSI = a (1 - exp(-b ISI))^c
// and build-up effect exp(50 ln(q) (1/BUI - 1/BUI0)), per fuel code.
// (Forestry Canada 1992 FBP System, with the 2009 updates; the paper cites it
// in Sections 1 and 2.3 without printing it.)  M-1/M-2 carry only (q, BUI0):
// their rates mix the C-2 and D-1 curves; M-3/M-4 carry their dead-fir
// curves, mixed with D-1 by percent dead fir.
#pragma once

// code:        a      b       c    q     BUI0
#define C2F_FUEL_ROWS                                                   \
    /*  0 non-fuel */ {0.0, 0.0, 0.0, 0.0, 0.0},                        \
    /*  1 C-1  */ {90.0, 0.0649, 4.5, 0.90, 72.0},                      \
    /*  2 C-2  */ {110.0, 0.0282, 1.5, 0.70, 64.0},                     \
    /*  3 C-3  */ {110.0, 0.0444, 3.0, 0.75, 62.0},                     \
    /*  4 C-4  */ {110.0, 0.0293, 1.5, 0.80, 66.0},                     \
    /*  5 C-5  */ {30.0, 0.0697, 4.0, 0.80, 56.0},                      \
    /*  6 C-6  */ {30.0, 0.0800, 3.0, 0.80, 62.0},                      \
    /*  7 C-7  */ {45.0, 0.0305, 2.0, 0.85, 106.0},                     \
    /*  8 D-1  */ {30.0, 0.0232, 1.6, 0.90, 32.0},                      \
    /*  9 M-1  */ {0.0, 0.0, 0.0, 0.80, 50.0},                          \
    /* 10 M-2  */ {0.0, 0.0, 0.0, 0.80, 50.0},                          \
    /* 11 S-1  */ {75.0, 0.0297, 1.3, 0.75, 38.0},                      \
    /* 12 S-2  */ {40.0, 0.0438, 1.7, 0.75, 63.0},                      \
    /* 13 S-3  */ {55.0, 0.0829, 3.2, 0.75, 31.0},                      \
    /* 14 O-1a */ {190.0, 0.0310, 1.4, 1.0, 1.0},                       \
    /* 15 O-1b */ {250.0, 0.0350, 1.7, 1.0, 1.0},                       \
    /* 16 D-2  */ {6.0, 0.0232, 1.6, 0.90, 32.0},                       \
    /* 17 M-3  */ {120.0, 0.0572, 1.4, 0.80, 50.0},                     \
    /* 18 M-4  */ {100.0, 0.0404, 1.48, 0.80, 50.0}

// Crown base height (m) and crown fuel load (kg/m^2) of the fuels that crown
// (conifers and mixedwoods); zero elsewhere.
// code:        CBH   CFL
#define C2F_CROWN_ROWS                                                  \
    /*  0 */ {0.0, 0.0}, /*  1 C-1 */ {2.0, 0.75}, /*  2 C-2 */ {3.0, 0.8},  \
    /*  3 C-3 */ {8.0, 1.15}, /*  4 C-4 */ {4.0, 1.2}, /*  5 C-5 */ {18.0, 1.2}, \
    /*  6 C-6 */ {7.0, 1.8}, /*  7 C-7 */ {10.0, 0.5}, /*  8 D-1 */ {0.0, 0.0}, \
    /*  9 M-1 */ {6.0, 0.8}, /* 10 M-2 */ {6.0, 0.8}, /* 11 S-1 */ {0.0, 0.0},  \
    /* 12 S-2 */ {0.0, 0.0}, /* 13 S-3 */ {0.0, 0.0}, /* 14 O-1a */ {0.0, 0.0}, \
    /* 15 O-1b */ {0.0, 0.0}, /* 16 D-2 */ {0.0, 0.0}, /* 17 M-3 */ {6.0, 0.8}, \
    /* 18 M-4 */ {6.0, 0.8}

namespace c2f {
struct FuelCoef {
    double a, b, c, q, bui0;
};
struct CrownCoef {
    double cbh, cfl;
};
constexpr double kGrassFuelLoad = 0.35;   // kg/m^2, O-1a and O-1b

enum FuelCode : int {
    kNonFuel = 0, kC1 = 1, kC2 = 2, kC3 = 3, kC4 = 4, kC5 = 5, kC6 = 6, kC7 = 7, kD1 = 8,
    kM1 = 9, kM2 = 10, kS1 = 11, kS2 = 12, kS3 = 13, kO1a = 14, kO1b = 15, kD2 = 16, kM3 = 17, kM4 = 18,
    kNumFuels = 19
};
}  // namespace c2f
