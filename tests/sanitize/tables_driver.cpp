// Host sanitizer driver for the binary128 table builder (gp_tables.cpp): every
// scheme, R = 1..3, ell/dx from 6 to 192 and sigma/dx 1.5..3, plus the
// adaptive-order tables. Built with -fsanitize=address,undefined by
// tests/test_host_sanitizers.py; exits non-zero on a non-finite table entry.
#include <cmath>
#include <cstdio>

#include "gp_tables.h"

static bool finite_all(const double* p, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int main() {
    const double ells[] = {6.0, 12.0, 24.0, 51.2, 80.0, 120.0, 192.0};
    const double sigmas[] = {1.5, 1.8, 3.0};
    int built = 0, refused = 0, bad = 0;
    for (int scheme = 0; scheme <= 2; ++scheme)
        for (int R = 1; R <= 3; ++R)
            for (double l : ells)
                for (double s : sigmas) {
                    GpTablesF64 t;
                    const int st = gpw_build_tables(scheme, R, l, s, &t);
                    if (st != 0) {
                        ++refused;
                        continue;
                    }
                    ++built;
                    if (!finite_all(&t.w_plus[0][0], 16) || !finite_all(&t.w_minus[0][0], 16) ||
                        !finite_all(t.gam_plus, 4) || !finite_all(&t.P[0][0][0], 64) ||
                        !finite_all(&t.gw_plus[0][0], 16) || !std::isfinite(t.mirror_residual))
                        ++bad;
                }
    for (double l : ells)
        for (double s : sigmas) {
            GpAoTablesF64 ao;
            if (gpw_build_ao_tables(l, s, &ao) == 0) {
                ++built;
                if (!finite_all(ao.w7_plus, 7) || !finite_all(&ao.P7[0][0], 49) || !finite_all(ao.c, 3)) ++bad;
            } else {
                ++refused;
            }
        }
    std::printf("tables built %d refused %d non-finite %d\n", built, refused, bad);
    return bad ? 1 : 0;
}
