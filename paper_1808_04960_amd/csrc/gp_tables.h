// Host-side pre-simulation tables (binary128 arithmetic, float64 results).
#pragma once

struct GpTablesF64 {
    double w_plus[4][4];   // [m][j]: sub-stencil m = 0..R, node j (offset m-R+j), x_* = +1/2
    double w_minus[4][4];  // same for x_* = -1/2
    double gam_plus[4];    // linear weights for x_* = +1/2
    double gam_minus[4];   // linear weights for x_* = -1/2
    double P[4][4][4];     // [m][i][j]: smoothness indicator beta_m = sum_i (P[m][i] . f_m)^2
    // GP indicators, R = 2 and 3: the same rows v_i / sqrt(lambda_i) written on
    // sums and differences of mirrored sub-stencil values. K(sigma) is symmetric
    // Toeplitz, so each eigenvector is symmetric or antisymmetric about the
    // sub-stencil centre. With s_j = f_j + f_{R-j} and d_j = f_j - f_{R-j}:
    //   R = 2: rows 0, 1: Ps[i][0] s_0 + Ps[i][1] f_1;  row 2: Ps[2][0] d_0;
    //   R = 3: rows 0, 1: Ps[i][0] s_0 + Ps[i][1] s_1;  rows 2, 3: Ps[i][0] d_0 + Ps[i][1] d_1.
    double Ps[4][2];
    double gw_plus[4][4];  // gam_plus[m] * w_plus[m][j], rounded once from binary128
    // largest relative difference between w_minus / gam_minus solved directly and
    // the mirror image of w_plus / gam_plus: zero in exact arithmetic, so it
    // measures how far the binary128 solves drift as K loses conditioning
    double mirror_residual;
};

// Interpolation schemes (values of gpweno_scheme).
enum { GPW_SCHEME_GP_WENO = 0, GPW_SCHEME_WENO_JS = 1, GPW_SCHEME_WENO_GP = 2, GPW_SCHEME_GP_AO = 3 };

// Extra tables of the adaptive-order GP interpolation (App. A of the paper):
// whole-stencil GP weights of radius 3 and 2, and for K_N(sigma), N = 7, 5, 3,
// the rows v_i / sqrt(lambda_i) and the constant N/2 log(2 pi) + 1/2 log det.
// The 3-point sub-stencil weights are GpTablesF64::w_plus / w_minus of R = 2.
struct GpAoTablesF64 {
    double w7_plus[7], w7_minus[7];
    double w5_plus[5], w5_minus[5];
    double P7[7][7], P5[5][5], P3[3][3];
    double c[3];           // N = 7, 5, 3
    double mirror_residual;  // as GpTablesF64::mirror_residual, for the 7- and 5-point weights
};

// Same return codes as gpw_build_tables (-4 does not occur).
int gpw_build_ao_tables(double ell_over_dx, double sigma_over_dx, GpAoTablesF64 *out);

// Returns 0 on success, < 0 on failure: -1 invalid input, -2 a failed weight
// solve, -3 a non-positive eigenvalue, -4 indicator rows in symmetric form that
// do not reproduce the eigen form, -5 weights of x_* = -1/2 that are not the
// mirror image of those of x_* = +1/2 (w_minus[m][j] = w_plus[R-m][R-j],
// gam_minus[m] = gam_plus[R-m]) to 1e-6, on which the sweep kernels rely (for
// R = 3 this also rejects ell beyond about 220-250 dx, where K is too badly
// conditioned for the binary128 solves to agree).
int gpw_build_tables(int scheme, int R, double ell_over_dx, double sigma_over_dx, GpTablesF64 *out);
