// Host-side pre-simulation tables (binary128 arithmetic, float64 results).
#pragma once

struct GpTablesF64 {
    double w_plus[4][4];   // [m][j]: sub-stencil m = 0..R, node j (offset m-R+j), x_* = +1/2
    double w_minus[4][4];  // same for x_* = -1/2
    double gam_plus[4];    // linear weights for x_* = +1/2
    double gam_minus[4];   // linear weights for x_* = -1/2
    double P[4][4];        // row i: v_i / sqrt(lambda_i) of K_m(sigma)
};

// Returns 0 on success, < 0 on invalid input or a failed factorisation.
int gpw_build_tables(int R, double ell_over_dx, double sigma_over_dx, GpTablesF64 *out);
