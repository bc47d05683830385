/* Host sanitizer driver for the CPU oracle (oracle/gpweno_oracle.c, included as
 * one translation unit): right-hand sides and steps for ndim 1..3, R 1..3, the
 * two- and three-term flux corrections, periodic, outflow and reflecting sides,
 * on small ragged grids, with simple averaging tables (memory safety only: the
 * values are not the scheme's). Built with -fsanitize=address,undefined by
 * tests/test_host_sanitizers.py; exits non-zero on a non-finite result. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/gpweno_oracle.c"

int main(void) {
    int runs = 0, bad = 0;
    const int sizes[3][3] = {{37, 1, 1}, {23, 17, 1}, {13, 11, 9}};
    for (int ndim = 1; ndim <= 3; ++ndim)
        for (int R = 1; R <= 3; ++R)
            for (int nc = 2; nc <= 3; ++nc)
                for (int bck = 0; bck <= 2; ++bck) {
                    oracle_cfg c;
                    memset(&c, 0, sizeof c);
                    c.ndim = ndim;
                    c.R = R;
                    c.gamma = 1.4;
                    c.flux_corr_terms = nc;
                    for (int d = 0; d < 3; ++d) {
                        c.n[d] = d < ndim ? sizes[ndim - 1][d] : 1;
                        c.dx[d] = 1.0 / c.n[d];
                        c.bc[d][0] = d < ndim ? bck : 0;
                        c.bc[d][1] = d < ndim ? bck : 0;
                        for (int m = 0; m <= R; ++m) {
                            c.gp[d][m] = c.gm[d][m] = 1.0 / (R + 1);
                            for (int j = 0; j <= R; ++j) {
                                c.wp[d][m][j] = c.wm[d][m][j] = 1.0 / (R + 1);
                                c.P[d][m][j] = m == j ? 1.0 : 0.0;
                            }
                        }
                    }
                    size_t ncell = (size_t)c.n[0] * c.n[1] * c.n[2];
                    int nv = 2 + ndim;
                    double *U = malloc(sizeof(double) * nv * ncell), *L = malloc(sizeof(double) * nv * ncell);
                    for (size_t i = 0; i < ncell; ++i) {
                        double rho = 1.0 + 0.1 * sin(0.37 * (double)i), u = 0.3 * cos(0.11 * (double)i);
                        U[i] = rho;
                        for (int d = 0; d < ndim; ++d) U[(1 + d) * ncell + i] = rho * u;
                        U[(nv - 1) * ncell + i] = 1.0 / 0.4 + 0.5 * rho * u * u * ndim;
                    }
                    oracle_rhs(&c, U, L);
                    double t = 0.0;
                    long n = 0;
                    oracle_run(&c, U, 0.4, 1e9, 2, &t, &n);
                    for (size_t i = 0; i < nv * ncell; ++i)
                        if (!isfinite(U[i]) || !isfinite(L[i])) {
                            ++bad;
                            break;
                        }
                    ++runs;
                    free(U);
                    free(L);
                }
    printf("oracle runs %d non-finite %d\n", runs, bad);
    return bad ? 1 : 0;
}
