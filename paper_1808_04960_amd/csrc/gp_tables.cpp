// Pre-simulation GP tables in binary128 (Sec. 4 step 1 of the paper).
//
//   (b) squared-exponential covariance K on the 2R+1 stencil and K_m on each
//       R+1 sub-stencil (Eq. (kmat)), prediction vectors k_* (Eq. (kstar)),
//       GP weights w^T = k_*^T K^{-1} (Sec. 3.2, Eq. (q-intrp));
//   (c) linear weights gamma: least-squares solution of M gamma = w_*
//       (Sec. 3.3, Eqs. (gamm-system), (M-mat));
//   (d) eigensystem of K_m built with sigma (Sec. 3.4); rows P_i = v_i/sqrt(lambda_i)
//       (Eq. (beta-eigen)).
//
// The same tables for the paper's comparison schemes (Sec. 6.2, Table
// (weno-vortex)): polynomial WENO interpolation (Lagrange weights on the
// sub-stencils and their linear weights) with either Jiang-Shu smoothness
// indicators (WENO-JS) or the GP ones (WENO-GP). Every scheme stores its
// smoothness indicator as beta_m = sum_i (P[m][i] . f_m)^2, so the sweep kernel
// is the same for all of them.
//
// K is badly conditioned at the usual ell = 12 dx (about 1e5, 6e9, 8e13 for
// R = 1, 2, 3, and far worse for larger ell/dx), so a float64 solve loses up to
// four digits of w for R = 3. Everything here runs in IEEE binary128 (113-bit
// significand) and is rounded to float64 once at the end.
//
// Coordinates are in units of dx: stencil nodes at the integers -R..R, the
// prediction point at x_* = +1/2 (w_plus) or -1/2 (w_minus).
// Built with g++ (binary128 arithmetic and expq/sqrtq from libquadmath).
#include <quadmath.h>

#include <cmath>
#include <cstring>
#include <utility>

#include "gp_tables.h"

namespace {

typedef __float128 q128;

constexpr int NMAX = 7;  // 2R+1 for R <= 3

q128 se_kernel(q128 a, q128 b, q128 ell) {
    q128 d = a - b;
    return expq(-(d * d) / (2 * ell * ell));
}

// Solve A x = b for symmetric positive definite A (n <= NMAX) by Cholesky.
bool cholesky_solve(int n, const q128 A[NMAX][NMAX], const q128 *b, q128 *x) {
    q128 L[NMAX][NMAX] = {};
    for (int j = 0; j < n; ++j) {
        q128 s = A[j][j];
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        if (!(s > 0)) return false;
        L[j][j] = sqrtq(s);
        for (int i = j + 1; i < n; ++i) {
            q128 t = A[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    q128 y[NMAX];
    for (int i = 0; i < n; ++i) {
        q128 t = b[i];
        for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
        y[i] = t / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {
        q128 t = y[i];
        for (int k = i + 1; k < n; ++k) t -= L[k][i] * x[k];
        x[i] = t / L[i][i];
    }
    return true;
}

// Least squares min ||A x - b|| for A (m x n, m >= n, full column rank) by
// Householder QR.
bool householder_lsq(int m, int n, q128 A[NMAX][NMAX], q128 *b, q128 *x) {
    for (int k = 0; k < n; ++k) {
        q128 norm = 0;
        for (int i = k; i < m; ++i) norm += A[i][k] * A[i][k];
        norm = sqrtq(norm);
        if (norm == 0) return false;
        q128 alpha = (A[k][k] > 0) ? -norm : norm;
        q128 v[NMAX] = {};
        for (int i = k; i < m; ++i) v[i] = A[i][k];
        v[k] -= alpha;
        q128 vv = 0;
        for (int i = k; i < m; ++i) vv += v[i] * v[i];
        if (vv == 0) continue;
        for (int j = k; j < n; ++j) {
            q128 s = 0;
            for (int i = k; i < m; ++i) s += v[i] * A[i][j];
            s = 2 * s / vv;
            for (int i = k; i < m; ++i) A[i][j] -= s * v[i];
        }
        q128 s = 0;
        for (int i = k; i < m; ++i) s += v[i] * b[i];
        s = 2 * s / vv;
        for (int i = k; i < m; ++i) b[i] -= s * v[i];
    }
    for (int i = n - 1; i >= 0; --i) {
        q128 t = b[i];
        for (int j = i + 1; j < n; ++j) t -= A[i][j] * x[j];
        if (A[i][i] == 0) return false;
        x[i] = t / A[i][i];
    }
    return true;
}

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (n <= M).
// On return A's diagonal holds the eigenvalues and V's columns the eigenvectors.
template <int M>
void jacobi_eigen(int n, q128 (&A)[M][M], q128 (&V)[M][M]) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i][j] = (i == j) ? 1 : 0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        q128 off = 0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[p][q] * A[p][q];
        if (off < (q128)1e-60 * (q128)1e-6) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                if (A[p][q] == 0) continue;
                q128 theta = (A[q][q] - A[p][p]) / (2 * A[p][q]);
                q128 t = (theta >= 0 ? 1 : -1) / (fabsq(theta) + sqrtq(theta * theta + 1));
                q128 c = 1 / sqrtq(t * t + 1);
                q128 s = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    q128 akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    q128 apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    q128 vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
        }
    }
}

// GP weights and linear weights for one prediction point x_*.
bool weights_for_point(int R, q128 ell, q128 xstar, q128 w[4][4], q128 gam[4]) {
    const int n = 2 * R + 1;
    q128 nodes[NMAX];
    for (int j = 0; j < n; ++j) nodes[j] = (q128)(j - R);
    // full stencil: K w_* = k_*
    q128 K[NMAX][NMAX], ks[NMAX], wstar[NMAX];
    for (int i = 0; i < n; ++i) {
        ks[i] = se_kernel(xstar, nodes[i], ell);
        for (int j = 0; j < n; ++j) K[i][j] = se_kernel(nodes[i], nodes[j], ell);
    }
    if (!cholesky_solve(n, K, ks, wstar)) return false;
    // sub-stencils m = 0..R over nodes m-R .. m
    for (int m = 0; m <= R; ++m) {
        q128 Km[NMAX][NMAX], km[NMAX], wm[NMAX];
        for (int i = 0; i <= R; ++i) {
            km[i] = ks[m + i];
            for (int j = 0; j <= R; ++j) Km[i][j] = K[m + i][m + j];
        }
        if (!cholesky_solve(R + 1, Km, km, wm)) return false;
        for (int j = 0; j <= R; ++j) w[m][j] = wm[j];
    }
    // M gamma = w_*, column m holds w_m in rows m..m+R
    q128 M[NMAX][NMAX] = {};
    for (int m = 0; m <= R; ++m)
        for (int j = 0; j <= R; ++j) M[m + j][m] = w[m][j];
    q128 rhs[NMAX], g[NMAX];
    for (int i = 0; i < n; ++i) rhs[i] = wstar[i];
    if (!householder_lsq(n, R + 1, M, rhs, g)) return false;
    for (int m = 0; m <= R; ++m) gam[m] = g[m];
    return true;
}

// Lagrange interpolation weights of the nodes x[0..n-1] at the point xs.
void lagrange_weights(int n, const q128 *x, q128 xs, q128 *w) {
    for (int j = 0; j < n; ++j) {
        q128 v = 1;
        for (int k = 0; k < n; ++k)
            if (k != j) v *= (xs - x[k]) / (x[j] - x[k]);
        w[j] = v;
    }
}

// Polynomial WENO interpolation weights and linear weights for one prediction
// point: the Lagrange limit of weights_for_point.
bool poly_weights_for_point(int R, q128 xstar, q128 w[4][4], q128 gam[4]) {
    const int n = 2 * R + 1;
    q128 nodes[NMAX], wstar[NMAX];
    for (int j = 0; j < n; ++j) nodes[j] = (q128)(j - R);
    lagrange_weights(n, nodes, xstar, wstar);
    for (int m = 0; m <= R; ++m) lagrange_weights(R + 1, nodes + m, xstar, w[m]);
    q128 M[NMAX][NMAX] = {};
    for (int m = 0; m <= R; ++m)
        for (int j = 0; j <= R; ++j) M[m + j][m] = w[m][j];
    q128 rhs[NMAX], g[NMAX];
    for (int i = 0; i < n; ++i) rhs[i] = wstar[i];
    if (!householder_lsq(n, R + 1, M, rhs, g)) return false;
    for (int m = 0; m <= R; ++m) gam[m] = g[m];
    return true;
}

// Jiang-Shu smoothness indicator of sub-stencil m (nodes m-R..m) as a quadratic
// form beta = f^T B f: B_ij = sum_{l=1..R} int_{-1/2}^{1/2} L_i^(l)(x) L_j^(l)(x) dx
// with L_j the Lagrange basis of the sub-stencil, unit spacing. The integrands
// have degree <= 2R-2 <= 4, so 3-point Gauss-Legendre quadrature is exact.
void js_form(int R, int m, q128 B[4][4]) {
    const int np = R + 1;
    q128 coef[4][4] = {};  // coef[j][k]: x^k coefficient of L_j
    for (int j = 0; j < np; ++j) {
        q128 c[4] = {1, 0, 0, 0};
        int deg = 0;
        const q128 xj = (q128)(m - R + j);
        for (int k = 0; k < np; ++k) {
            if (k == j) continue;
            const q128 xk = (q128)(m - R + k);
            const q128 s = 1 / (xj - xk);
            q128 nc[4] = {0, 0, 0, 0};  // c * (x - xk) * s
            for (int a = 0; a <= deg; ++a) {
                nc[a + 1] += c[a] * s;
                nc[a] -= c[a] * xk * s;
            }
            ++deg;
            for (int a = 0; a < 4; ++a) c[a] = nc[a];
        }
        for (int a = 0; a < 4; ++a) coef[j][a] = c[a];
    }
    const q128 g = sqrtq((q128)3 / 5) / 2;
    const q128 qx[3] = {-g, 0, g};
    const q128 qw[3] = {(q128)5 / 18, (q128)8 / 18, (q128)5 / 18};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) B[i][j] = 0;
    for (int l = 1; l <= R; ++l) {
        for (int q = 0; q < 3; ++q) {
            q128 d[4];
            for (int j = 0; j < np; ++j) {  // l-th derivative of L_j at qx[q]
                q128 v = 0;
                for (int k = l; k < np; ++k) {
                    q128 fall = 1;
                    for (int t = 0; t < l; ++t) fall *= (q128)(k - t);
                    v += coef[j][k] * fall * powq(qx[q], k - l);
                }
                d[j] = v;
            }
            for (int i = 0; i < np; ++i)
                for (int j = 0; j < np; ++j) B[i][j] += qw[q] * d[i] * d[j];
        }
    }
}

// GP weights of the whole stencil of radius R at x_* (Eq. (q-intrp)).
bool full_weights(int R, q128 ell, q128 xstar, q128 *w) {
    const int n = 2 * R + 1;
    q128 K[NMAX][NMAX], ks[NMAX];
    for (int i = 0; i < n; ++i) {
        ks[i] = se_kernel(xstar, (q128)(i - R), ell);
        for (int j = 0; j < n; ++j) K[i][j] = se_kernel((q128)(i - R), (q128)(j - R), ell);
    }
    return cholesky_solve(n, K, ks, w);
}

// Rows v_i / sqrt(lambda_i) of K_N(sigma) on N consecutive nodes, and
// N/2 log(2 pi) + 1/2 log det K_N(sigma) (the sum of the log eigenvalues).
bool kernel_rows(int N, q128 sig, double *P /* [N][N] */, double *cN) {
    q128 A[NMAX][NMAX] = {}, V[NMAX][NMAX] = {};
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) A[i][j] = se_kernel((q128)i, (q128)j, sig);
    jacobi_eigen(N, A, V);
    q128 logdet = 0;
    for (int i = 0; i < N; ++i) {
        const q128 lam = A[i][i];
        if (!(lam > 0)) return false;
        logdet += logq(lam);
        const q128 inv = 1 / sqrtq(lam);
        for (int j = 0; j < N; ++j) P[N * i + j] = (double)(V[j][i] * inv);
    }
    const q128 pi = 4 * atanq((q128)1);
    *cN = (double)((q128)N / 2 * logq(2 * pi) + logdet / 2);
    return true;
}

// The weights of x_* = -1/2 are those of x_* = +1/2 mirrored about the centre
// node: K and the stencil set are symmetric under x -> -x, which maps node j of
// sub-stencil m to node R - j of sub-stencil R - m. The sweep kernels read only
// the +1/2 set; this checks the identity on the two binary128 solves. A defect
// would break it by O(1); the solves themselves drift apart as K loses
// conditioning (R = 3 linear weights and 7-point weights: 1e-12 at ell = 80 dx,
// 7e-8 at 192 dx, 2e-3 at 400 dx, where the tables no longer hold any digits
// worth using), so the tolerance is 1e-6 relative.
constexpr double MIRROR_TOL = 1e-6;

// Largest relative difference between the two solves: |w_- - mirror(w_+)| over
// the largest |w_+| of one stencil of n nodes.
q128 mirror_residual(int n, const q128 *wp, const q128 *wm) {
    q128 scale = 0, r = 0;
    for (int j = 0; j < n; ++j) scale = fmaxq(scale, fabsq(wp[j]));
    for (int j = 0; j < n; ++j) r = fmaxq(r, fabsq(wm[j] - wp[n - 1 - j]) / scale);
    return r;
}

// The same over every sub-stencil's weights (relative to the largest |w_+|) and
// the linear weights (absolute: the gammas sum to about 1).
q128 mirror_residual(int R, const q128 wp[4][4], const q128 wm[4][4], const q128 *gp, const q128 *gm) {
    q128 scale = 0, r = 0;
    for (int m = 0; m <= R; ++m)
        for (int j = 0; j <= R; ++j) scale = fmaxq(scale, fabsq(wp[m][j]));
    for (int m = 0; m <= R; ++m) {
        r = fmaxq(r, fabsq(gm[m] - gp[R - m]));
        for (int j = 0; j <= R; ++j) r = fmaxq(r, fabsq(wm[m][j] - wp[R - m][R - j]) / scale);
    }
    return r;
}

}  // namespace

int gpw_build_ao_tables(double ell_over_dx, double sigma_over_dx, GpAoTablesF64 *out) {
    if (!(ell_over_dx > 0) || !(sigma_over_dx > 0) || !out) return -1;
    std::memset(out, 0, sizeof(*out));
    const q128 ell = (q128)ell_over_dx, sig = (q128)sigma_over_dx;
    q128 w7p[NMAX], w7m[NMAX], w5p[NMAX], w5m[NMAX];
    if (!full_weights(3, ell, (q128)0.5, w7p) || !full_weights(3, ell, (q128)-0.5, w7m)) return -2;
    if (!full_weights(2, ell, (q128)0.5, w5p) || !full_weights(2, ell, (q128)-0.5, w5m)) return -2;
    const q128 res = fmaxq(mirror_residual(7, w7p, w7m), mirror_residual(5, w5p, w5m));
    if (!(res <= (q128)MIRROR_TOL)) return -5;
    out->mirror_residual = (double)res;
    for (int j = 0; j < 7; ++j) {
        out->w7_plus[j] = (double)w7p[j];
        out->w7_minus[j] = (double)w7m[j];
    }
    for (int j = 0; j < 5; ++j) {
        out->w5_plus[j] = (double)w5p[j];
        out->w5_minus[j] = (double)w5m[j];
    }
    if (!kernel_rows(7, sig, &out->P7[0][0], &out->c[0])) return -3;
    if (!kernel_rows(5, sig, &out->P5[0][0], &out->c[1])) return -3;
    if (!kernel_rows(3, sig, &out->P3[0][0], &out->c[2])) return -3;
    return 0;
}

// GP indicator rows of K(sigma) on R + 1 = 3 or 4 nodes in symmetric /
// antisymmetric form (GpTablesF64::Ps). In the orthonormal basis of mirrored
// sums and differences, K splits into a symmetric and an antisymmetric block,
// each diagonalised here; the eigenvectors of K are those of the blocks mapped
// back, so the rows are the v_i / sqrt(lambda_i) of the eigen form, each
// symmetric or antisymmetric by construction. K[i][j] = k[|i - j|].
bool symmetric_rows(int R, const q128 *k, double Ps[4][2]) {
    const q128 r2 = sqrtq((q128)2);
    // blocks in the bases {(e_0 + e_R)/sqrt2, centre or (e_1 + e_{R-1})/sqrt2} and
    // {(e_0 - e_R)/sqrt2, (e_1 - e_{R-1})/sqrt2}
    q128 S[2][2], A[2][2];
    int na;
    if (R == 2) {
        S[0][0] = k[0] + k[2];
        S[0][1] = S[1][0] = r2 * k[1];
        S[1][1] = k[0];
        A[0][0] = k[0] - k[2];
        na = 1;
    } else if (R == 3) {
        S[0][0] = k[0] + k[3];
        S[0][1] = S[1][0] = k[1] + k[2];
        S[1][1] = k[0] + k[1];
        A[0][0] = k[0] - k[3];
        A[0][1] = A[1][0] = k[1] - k[2];
        A[1][1] = k[0] - k[1];
        na = 2;
    } else {
        return false;
    }
    q128 VS[2][2], VA[2][2];
    jacobi_eigen(2, S, VS);
    jacobi_eigen(na, A, VA);
    for (int i = 0; i < 2; ++i) {
        if (!(S[i][i] > 0)) return false;
        const q128 f = 1 / sqrtq(S[i][i]);
        // R = 2: the centre basis vector is e_1 itself (no 1/sqrt2)
        Ps[i][0] = (double)(VS[0][i] * f / r2);
        Ps[i][1] = (double)(VS[1][i] * f / (R == 2 ? (q128)1 : r2));
    }
    for (int i = 0; i < na; ++i) {
        if (!(A[i][i] > 0)) return false;
        const q128 f = 1 / sqrtq(A[i][i]);
        Ps[2 + i][0] = (double)(VA[0][i] * f / r2);
        Ps[2 + i][1] = na == 2 ? (double)(VA[1][i] * f / r2) : 0.0;
    }
    return true;
}

// beta = f^T K^{-1} f from the eigen rows P and from the symmetric rows Ps, for
// a fixed set of test vectors; true if they agree to the rounding of the
// float64 rows, measured on the scale sum_i (sum_j |P_ij f_j|)^2 (beta itself
// can be far smaller when K is badly conditioned). A wrong sign or row gives an
// error of the order of that scale.
bool symmetric_rows_agree(int R, const double (*P)[4], const double Ps[4][2]) {
    const double tests[4][4] = {{1.0, -0.5, 0.25, 2.0}, {0.3, 0.3, 0.3, 0.3}, {-1.0, 2.0, -1.0, 0.5}, {0.0, 1e-3, 2e-3, 3e-3}};
    for (const auto &f : tests) {
        q128 b1 = 0, b2 = 0, scale = 0;
        for (int i = 0; i <= R; ++i) {
            q128 p = 0, pa = 0;
            for (int j = 0; j <= R; ++j) {
                p += (q128)P[i][j] * f[j];
                pa += fabsq((q128)P[i][j] * f[j]);
            }
            b1 += p * p;
            scale += pa * pa;
        }
        const q128 s0 = (q128)f[0] + f[R], d0 = (q128)f[0] - f[R];
        const q128 s1 = R == 2 ? (q128)f[1] : (q128)f[1] + f[2], d1 = R == 2 ? (q128)0 : (q128)f[1] - f[2];
        for (int i = 0; i < 2; ++i) {
            const q128 p = Ps[i][0] * s0 + Ps[i][1] * s1;
            b2 += p * p;
        }
        for (int i = 2; i <= R; ++i) {
            const q128 p = Ps[i][0] * d0 + Ps[i][1] * d1;
            b2 += p * p;
        }
        if (!(fabsq(b1 - b2) <= (q128)1e-12 * scale)) return false;
    }
    return true;
}

int gpw_build_tables(int scheme, int R, double ell_over_dx, double sigma_over_dx, GpTablesF64 *out) {
    if (R < 1 || R > 3 || !(ell_over_dx > 0) || !(sigma_over_dx > 0) || !out) return -1;
    if (scheme != GPW_SCHEME_GP_WENO && scheme != GPW_SCHEME_WENO_JS && scheme != GPW_SCHEME_WENO_GP) return -1;
    if (scheme == GPW_SCHEME_WENO_JS && R > 2) return -1;
    std::memset(out, 0, sizeof(*out));
    q128 wp[4][4] = {}, wm[4][4] = {}, gp[4] = {}, gm[4] = {};
    if (scheme == GPW_SCHEME_GP_WENO) {
        const q128 ell = (q128)ell_over_dx;
        if (!weights_for_point(R, ell, (q128)0.5, wp, gp)) return -2;
        if (!weights_for_point(R, ell, (q128)-0.5, wm, gm)) return -2;
    } else {
        if (!poly_weights_for_point(R, (q128)0.5, wp, gp)) return -2;
        if (!poly_weights_for_point(R, (q128)-0.5, wm, gm)) return -2;
    }
    const q128 res = mirror_residual(R, wp, wm, gp, gm);
    if (!(res <= (q128)MIRROR_TOL)) return -5;
    if (scheme == GPW_SCHEME_WENO_JS) {
        // factor each B_m = V diag(lambda) V^T; rows sqrt(lambda_i) v_i in order of
        // decreasing lambda. B_m is positive semi-definite of rank R (its null
        // space is the constants), so row R is zero and the sweep skips it.
        for (int m = 0; m <= R; ++m) {
            q128 A[4][4], V[4][4] = {};
            js_form(R, m, A);
            jacobi_eigen(R + 1, A, V);
            int order[4] = {0, 1, 2, 3};
            for (int a = 0; a <= R; ++a)
                for (int b = a + 1; b <= R; ++b)
                    if (A[order[b]][order[b]] > A[order[a]][order[a]]) std::swap(order[a], order[b]);
            for (int i = 0; i <= R; ++i) {
                const q128 lam = A[order[i]][order[i]];
                const q128 s = (i < R && lam > 0) ? sqrtq(lam) : (q128)0;
                for (int j = 0; j <= R; ++j) out->P[m][i][j] = (double)(V[j][order[i]] * s);
            }
        }
    } else {
        // eigensystem of K_m(sigma) on nodes 0..R (identical for every sub-stencil)
        const q128 sig = (q128)sigma_over_dx;
        q128 A[4][4] = {}, V[4][4] = {};
        for (int i = 0; i <= R; ++i)
            for (int j = 0; j <= R; ++j) A[i][j] = se_kernel((q128)i, (q128)j, sig);
        jacobi_eigen(R + 1, A, V);
        for (int i = 0; i <= R; ++i) {
            const q128 lam = A[i][i];
            if (!(lam > 0)) return -3;
            const q128 inv = 1 / sqrtq(lam);
            for (int j = 0; j <= R; ++j) {
                const double v = (double)(V[j][i] * inv);
                for (int m = 0; m <= R; ++m) out->P[m][i][j] = v;
            }
        }
        if (R >= 2) {
            q128 k[4];
            for (int t = 0; t <= R; ++t) k[t] = se_kernel((q128)0, (q128)t, sig);
            if (!symmetric_rows(R, k, out->Ps)) return -3;
            if (!symmetric_rows_agree(R, out->P[0], out->Ps)) return -4;
        }
    }
    for (int m = 0; m <= R; ++m) {
        out->gam_plus[m] = (double)gp[m];
        out->gam_minus[m] = (double)gm[m];
        for (int j = 0; j <= R; ++j) {
            out->w_plus[m][j] = (double)wp[m][j];
            out->w_minus[m][j] = (double)wm[m][j];
            out->gw_plus[m][j] = (double)(gp[m] * wp[m][j]);
        }
    }
    out->mirror_residual = (double)res;
    return 0;
}
