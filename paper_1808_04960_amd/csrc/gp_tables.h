// Host-side pre-simulation tables (binary128 arithmetic, float64 results).
#pragma once

struct GpTablesF64 {
    double w_plus[4][4];   // [m][j]: sub-stencil m = 0..R, node j (offset m-R+j), x_* = +1/2
    double w_minus[4][4];  // same for x_* = -1/2
    double gam_plus[4];    // linear weights for x_* = +1/2
    double gam_minus[4];   // linear weights for x_* = -1/2
    double P[4][4][4];     // [m][i][j]: smoothness indicator beta_m = sum_i (P[m][i] . f_m)^2
};

// Interpolation schemes (values of gpweno_scheme).
enum { GPW_SCHEME_GP_WENO = 0, GPW_SCHEME_WENO_JS = 1, GPW_SCHEME_WENO_GP = 2 };

// Returns 0 on success, < 0 on invalid input or a failed factorisation.
int gpw_build_tables(int scheme, int R, double ell_over_dx, double sigma_over_dx, GpTablesF64 *out);
