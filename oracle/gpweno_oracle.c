/*
 * CPU oracle for the GP-WENO finite-difference (FD-Prim) scheme for the
 * compressible Euler equations on uniform grids (periodic, outflow or
 * reflecting boundaries per axis side).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
 * GPU library is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product path never does, and this
 * file shares no code, header or table generator with the GPU library.
 *
 * Plain scalar float64, no blocking or fusion: every step is written in the
 * order the paper gives it.
 *   - Sec. 2, Eq. (disc_fd):          dU_i/dt = -(fhat_{i+1/2} - fhat_{i-1/2})/dx - ...
 *   - Sec. 2, Eq. (riemann_prob):     face flux F_{i+1/2} = RP(U^L, U^R)
 *   - Sec. 2, Eqs. (numFlux_cor), (FD-ders): fhat = F + alpha dx^2 F'' + beta dx^4 F''''
 *                                     with alpha = -1/24, beta = 3/640, no limiter;
 *                                     optionally the next term of the series, -5/7168
 *                                     on the sixth difference (the "+ ..." there)
 *   - Sec. 3.3, Eqs. (candidate_interp), (weight_sum), (weights), (gp-smooth),
 *     (beta-eigen):                   GP-WENO interpolation of the Riemann states
 *   - Sec. 4:                         stepwise algorithm
 *   - Sec. 7 (intro):                 characteristic variables, SSP-RK3, HLLC
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - primitive variables are projected onto the eigenvectors of the primitive
 *     Jacobian evaluated at the stencil-centre cell i; the same projection serves
 *     both Riemann states x_{i+-1/2} of that cell;
 *   - HLLC with Davis wave-speed estimates S_L = min(u_L-c_L, u_R-c_R),
 *     S_R = max(u_L+c_L, u_R+c_R); at S* = 0 the left star state is taken;
 *   - dt = CFL / max_i sum_d (|u_d| + c)/dx_d from the state at the start of the
 *     step, clipped so that t does not pass t_final;
 *   - SSP-RK3 in Shu-Osher form;
 *   - optional positivity fallback (off unless requested): a Riemann state with
 *     rho <= 0 or p <= 0 is replaced by the cell-centre primitive state.
 *
 * Layout of the state: conserved variables, structure of arrays
 * [nv][nz][ny][nx] with x fastest, nv = 2 + ndim:
 * (rho, rho u[, rho v[, rho w]], E).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define NVMAX 5
#define RMAX 3

typedef struct {
    int ndim;
    int n[3];
    double dx[3];
    int R;
    double gamma;           /* ratio of specific heats */
    int positivity_fallback;
    /* GP tables per direction, sub-stencil index first: [d][m][j] */
    double wp[3][4][4];     /* w_m at x_* = +1/2 */
    double wm[3][4][4];     /* w_m at x_* = -1/2 */
    double gp[3][4];        /* gamma_m for x_* = +1/2 */
    double gm[3][4];        /* gamma_m for x_* = -1/2 */
    double P[3][4][4];      /* rows P_i = v_i / sqrt(lambda_i) of K_m(sigma) */
    int beta_form;          /* 0: beta_m = sum_i (P_i . f_m)^2 (GP, Eq. (beta-eigen));
                               1: beta_m = f_m^T B_m f_m (polynomial, Jiang-Shu type) */
    double B[3][4][4][4];   /* [d][m][i][j], used when beta_form = 1 */
    int bc[3][2];           /* boundary kind per axis and side (0 low, 1 high):
                               0 periodic, 1 outflow, 2 reflecting wall */
    int nonzero_mean;       /* 1: GP indicators of f_m - f_i (centre-cell mean, Sec. 7) */
    /* adaptive-order GP (App. A); used when ao = 1: R = 3 gives GP-AO(3,2,3),
     * R = 2 gives GP-AO(2,3). side 0 is x_* = +1/2, side 1 is x_* = -1/2. */
    int ao;
    double ao_w7[3][2][7];      /* GP weights, 7-point stencil */
    double ao_w5[3][2][5];      /* GP weights, 5-point stencil */
    double ao_w3[3][2][3][3];   /* GP weights of the 3-point sub-stencils [m][j] */
    double ao_P7[3][7][7];      /* rows v_i / sqrt(lambda_i) of K_7(sigma) */
    double ao_P5[3][5][5];
    double ao_P3[3][3][3];
    double ao_c[3][3];          /* N/2 log 2pi + 1/2 log det K_N(sigma), N = 7, 5, 3 */
    double ao_gam[4];           /* CWENO linear weights gamma_1..3, then gamma_HI */
    int flux_corr_terms;        /* 2: alpha, beta (the paper's); 3: also the sixth
                                   difference; 0 reads as 2 */
} oracle_cfg;

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2 };

/* Primitive vector in a frame rotated to direction d:
 * (rho, u_n, u_t1, u_t2, p); absent velocity components are zero. */
enum { Q_RHO = 0, Q_UN = 1, Q_UT1 = 2, Q_UT2 = 3, Q_P = 4 };

/* Characteristic fields of the primitive Jacobian, in wave order. */
enum { K_ACM = 0, K_ENT = 1, K_T1 = 2, K_T2 = 3, K_ACP = 4 };

static const double EPS_WENO = 1e-36;   /* epsilon of Eq. (weights) */
static const double ALPHA_FC = -1.0 / 24.0;   /* Eq. (numFlux_cor) */
static const double BETA_FC = 3.0 / 640.0;
/* Next term of the same series: the numerical flux h whose difference gives the
 * derivative of F exactly, h = F - dx^2/24 F'' + 7 dx^4/5760 F'''' - 31 dx^6/967680
 * F^(6) + ..., with the derivatives written as central differences of the face
 * fluxes, gives -1/24 on the second, 3/640 on the fourth and -5/7168 on the
 * sixth difference. */
static const double C6_FC = -5.0 / 7168.0;

/* Active characteristic fields for a given dimension (nv of them). */
static int active_fields(int ndim, int *k) {
    if (ndim == 1) { k[0] = K_ACM; k[1] = K_ENT; k[2] = K_ACP; return 3; }
    if (ndim == 2) { k[0] = K_ACM; k[1] = K_ENT; k[2] = K_T1; k[3] = K_ACP; return 4; }
    k[0] = K_ACM; k[1] = K_ENT; k[2] = K_T1; k[3] = K_T2; k[4] = K_ACP; return 5;
}

/* Velocity component (0=x,1=y,2=z) that plays the role of n, t1, t2 for direction d. */
static void frame_axes(int d, int ax[3]) {
    if (d == 0) { ax[0] = 0; ax[1] = 1; ax[2] = 2; }
    else if (d == 1) { ax[0] = 1; ax[1] = 0; ax[2] = 2; }
    else { ax[0] = 2; ax[1] = 0; ax[2] = 1; }
}

static size_t ncells_of(const oracle_cfg *c) {
    size_t n = 1;
    for (int d = 0; d < c->ndim; ++d) n *= (size_t)c->n[d];
    return n;
}

/* ---------------------------------------------------------------------------
 * Euler system, Sec. 2 Eq. (euler).
 * ------------------------------------------------------------------------- */

/* Conserved (nv comps, cell-major view) -> primitive (rho, u, v, w, p) in xyz. */
void oracle_cons_to_prim(int ndim, double gamma, const double *u, double *v5) {
    int nv = 2 + ndim;
    double rho = u[0];
    double vel[3] = {0.0, 0.0, 0.0};
    double ke = 0.0;
    for (int d = 0; d < ndim; ++d) {
        vel[d] = u[1 + d] / rho;
        ke += vel[d] * u[1 + d];
    }
    v5[0] = rho;
    v5[1] = vel[0];
    v5[2] = vel[1];
    v5[3] = vel[2];
    v5[4] = (gamma - 1.0) * (u[nv - 1] - 0.5 * ke);
}

/* Physical flux in the rotated frame: (rho u_n, rho u_n^2 + p, rho u_n u_t1,
 * rho u_n u_t2, u_n (E + p)), E = p/(gamma-1) + rho |u|^2 / 2. */
static void phys_flux(const double *q, double gamma, double *F, double *Ucons) {
    double rho = q[Q_RHO], un = q[Q_UN], t1 = q[Q_UT1], t2 = q[Q_UT2], p = q[Q_P];
    double E = p / (gamma - 1.0) + 0.5 * rho * (un * un + t1 * t1 + t2 * t2);
    F[0] = rho * un;
    F[1] = rho * un * un + p;
    F[2] = rho * un * t1;
    F[3] = rho * un * t2;
    F[4] = un * (E + p);
    if (Ucons) {
        Ucons[0] = rho;
        Ucons[1] = rho * un;
        Ucons[2] = rho * t1;
        Ucons[3] = rho * t2;
        Ucons[4] = E;
    }
}

/* ---------------------------------------------------------------------------
 * Adaptive-order GP interpolation (App. A) of one variable to x_{i+1/2}
 * (side 0) or x_{i-1/2} (side 1), data f[0..2Rhi] = q_{i-Rhi} .. q_{i+Rhi},
 * Rhi = 3 (GP-AO(3,2,3)) or 2 (GP-AO(2,3)).
 *   smoothness indicators: the negative log-likelihood of Eq. (log-like) with
 *     zero mean, keeping its normalisation and complexity terms because the
 *     stencils differ in size: beta = c_N + 1/2 f^T K_N(sigma)^-1 f,
 *     with f^T K^-1 f = sum_i (P_i . f)^2 (Eq. (beta-eigen));
 *   GP-CWENO on the three 3-point sub-stencils of the 5-point stencil with the
 *     linear weights of Eq. (CWENO-lin);
 *   GP-AO(R,3), Eqs. (nonlin-AO), (GP-AO): weights gamma_HI/(eps+beta^R)^2 and
 *     gamma_m/(eps+beta_m)^2 normalised together, then
 *     q = omega^R/gamma_HI q^R + sum_m (omega_m - omega^R gamma_m/gamma_HI) q^m;
 *   GP-AO(R',R,3), Eqs. (recursive-weights), (AO-recursive): weights
 *     gamma_HI/(eps+beta^R')^2 and (1-gamma_HI)/(eps+beta^R)^2, normalised, then
 *     q = nu^R'/gamma_HI q^AO(R',3) + (nu^R - nu^R'(1-gamma_HI)/gamma_HI) q^AO(R,3).
 * Reading: the weights of the sub-stencils use gamma_m (the printed formula
 * repeats gamma_HI there, which would remove the bias towards the centred
 * stencil that the text describes).
 * ------------------------------------------------------------------------- */
static double quad_rows(int N, const double *P, const double *f) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) {
        double pr = 0.0;
        for (int j = 0; j < N; ++j) pr += P[N * i + j] * f[j];
        s += pr * pr;
    }
    return s;
}

static double dot(int N, const double *w, const double *f) {
    double s = 0.0;
    for (int j = 0; j < N; ++j) s += w[j] * f[j];
    return s;
}

/* GP-AO(R,3) from the high-order interpolation qR with indicator bR, and the
 * sub-stencil interpolations qm[3] with indicators bm[3]; gam = gamma_1..3,
 * gamma_HI (Eqs. (nonlin-AO), (GP-AO)). */
double oracle_ao_hybrid(double qR, double bR, const double *qm, const double *bm, const double *gam) {
    double ghi = gam[3];
    double wR = ghi / ((EPS_WENO + bR) * (EPS_WENO + bR));
    double wm[3], sum = wR;
    for (int m = 0; m < 3; ++m) {
        wm[m] = gam[m] / ((EPS_WENO + bm[m]) * (EPS_WENO + bm[m]));
        sum += wm[m];
    }
    double oR = wR / sum;
    double q = oR / ghi * qR;
    for (int m = 0; m < 3; ++m) q += (wm[m] / sum - oR / ghi * gam[m]) * qm[m];
    return q;
}

/* GP-AO(R',R,3) from GP-AO(R',3) and GP-AO(R,3) with the indicators of the
 * stencils S_R' and S_R (Eqs. (recursive-weights), (AO-recursive)). */
double oracle_ao_recursive(double aoHi, double bHi, double aoLo, double bLo, double ghi) {
    double nh = ghi / ((EPS_WENO + bHi) * (EPS_WENO + bHi));
    double nl = (1.0 - ghi) / ((EPS_WENO + bLo) * (EPS_WENO + bLo));
    double nuH = nh / (nh + nl), nuL = nl / (nh + nl);
    return nuH / ghi * aoHi + (nuL - nuH * (1.0 - ghi) / ghi) * aoLo;
}

void oracle_gp_ao(int Rhi, const double *f, const double *w7, const double *w5, const double *w3,
                  const double *P7, const double *P5, const double *P3, const double *cN,
                  const double *gam, double *q_out, double *beta_out) {
    const double *f5 = f + (Rhi - 2);           /* the 5-point stencil, nodes -2..2 */
    double b5 = cN[1] + 0.5 * quad_rows(5, P5, f5);
    double bm[3], qm[3];
    for (int m = 0; m < 3; ++m) {
        bm[m] = cN[2] + 0.5 * quad_rows(3, P3, f5 + m);
        qm[m] = dot(3, w3 + 3 * m, f5 + m);
    }
    double q5 = dot(5, w5, f5);
    double ao5 = oracle_ao_hybrid(q5, b5, qm, bm, gam);
    if (beta_out) {
        beta_out[1] = b5;
        for (int m = 0; m < 3; ++m) beta_out[2 + m] = bm[m];
    }
    if (Rhi == 2) {
        *q_out = ao5;
        return;
    }
    double b7 = cN[0] + 0.5 * quad_rows(7, P7, f);
    double q7 = dot(7, w7, f);
    double ao7 = oracle_ao_hybrid(q7, b7, qm, bm, gam);
    if (beta_out) beta_out[0] = b7;
    *q_out = oracle_ao_recursive(ao7, b7, ao5, b5, gam[3]);
}

/* ---------------------------------------------------------------------------
 * Characteristic decomposition (Sec. 7 intro: interpolation on characteristic
 * variables). Left rows l_k and right columns r_k of the primitive Jacobian in
 * the rotated frame, evaluated at q:
 *   l_acm = (0, -rho/(2c), 0, 0, 1/(2c^2)),  r_acm = (1, -c/rho, 0, 0, c^2)
 *   l_ent = (1, 0, 0, 0, -1/c^2),            r_ent = (1, 0, 0, 0, 0)
 *   l_t1  = e_{u_t1},  l_t2 = e_{u_t2}        r_t1, r_t2 the same unit vectors
 *   l_acp = (0, rho/(2c), 0, 0, 1/(2c^2)),   r_acp = (1, c/rho, 0, 0, c^2)
 * so that L R = I.
 * ------------------------------------------------------------------------- */
void oracle_char_vectors(const double *q, double gamma, double *Lm, double *Rm) {
    double rho = q[Q_RHO], p = q[Q_P];
    double c = sqrt(gamma * p / rho);
    double L[5][5], Rv[5][5];
    memset(L, 0, sizeof L);
    memset(Rv, 0, sizeof Rv);
    L[K_ACM][Q_UN] = -rho / (2.0 * c);
    L[K_ACM][Q_P] = 1.0 / (2.0 * c * c);
    L[K_ENT][Q_RHO] = 1.0;
    L[K_ENT][Q_P] = -1.0 / (c * c);
    L[K_T1][Q_UT1] = 1.0;
    L[K_T2][Q_UT2] = 1.0;
    L[K_ACP][Q_UN] = rho / (2.0 * c);
    L[K_ACP][Q_P] = 1.0 / (2.0 * c * c);
    /* right eigenvectors stored as Rv[k][component] (column k of R) */
    Rv[K_ACM][Q_RHO] = 1.0; Rv[K_ACM][Q_UN] = -c / rho; Rv[K_ACM][Q_P] = c * c;
    Rv[K_ENT][Q_RHO] = 1.0;
    Rv[K_T1][Q_UT1] = 1.0;
    Rv[K_T2][Q_UT2] = 1.0;
    Rv[K_ACP][Q_RHO] = 1.0; Rv[K_ACP][Q_UN] = c / rho; Rv[K_ACP][Q_P] = c * c;
    memcpy(Lm, L, sizeof L);
    memcpy(Rm, Rv, sizeof Rv);
}

/* ---------------------------------------------------------------------------
 * GP-WENO interpolation of one variable to x_{i+1/2} and x_{i-1/2}
 * (Sec. 3.3 and Sec. 4 step 2), data f[0..2R] = q_{i-R} .. q_{i+R}.
 *   candidate predictions   q^m_* = w_m^T f_m                     Eq. (candidate_interp)
 *   smoothness indicators   beta_m = sum_i (P_i . f_m)^2          Eq. (beta-eigen)
 *                           ( = f_m^T K_m^{-1} f_m, Eq. (gp-smooth), zero mean )
 *   nonlinear weights       w~_m = gamma_m / (eps + beta_m)^2,  omega = w~ / sum w~
 *                                                                 Eq. (weights), p = 2, eps = 1e-36
 *   result                  q_* = sum_m omega_m q^m_*             Eq. (weight_sum)
 * Sub-stencil m = 0..R holds f[m .. m+R]. beta is shared by the two
 * prediction points because the sub-stencils are the same sets.
 * Optional outputs (may be NULL): beta[R+1], omega_p[R+1], omega_m[R+1].
 * nonzero_mean: the GP indicator of f_m - f_i instead of f_m, with f_i = f[R]
 * the centre cell's value (Sec. 7, the non-zero-mean prior of the scalar
 * advection test).
 *
 * The same function serves the paper's comparison schemes (Sec. 6.2, Table
 * (weno-vortex)) with other tables: polynomial (Lagrange) weights and linear
 * weights in w and gamma, and, when B is given, the polynomial smoothness
 * indicator beta_m = f_m^T B_m f_m of the Jiang-Shu type (sum over derivative
 * orders of the squared derivatives of the interpolant, integrated over the
 * centre cell) in place of the GP one. The weight formula is unchanged.
 * ------------------------------------------------------------------------- */
void oracle_gp_weno(int R, const double *f,
                    const double *wp, const double *wm,   /* [4][4] */
                    const double *gp, const double *gm,   /* [4] */
                    const double *P,                      /* [4][4] */
                    const double *B,                      /* [4][4][4] or NULL */
                    int nonzero_mean,
                    double *qplus, double *qminus,
                    double *beta_out, double *omp_out, double *omm_out) {
    double beta[RMAX + 1], qp[RMAX + 1], qm[RMAX + 1];
    double wtp[RMAX + 1], wtm[RMAX + 1];
    double sp = 0.0, sm = 0.0;
    for (int m = 0; m <= R; ++m) {
        const double *fm = f + m;
        double b = 0.0;
        if (B) {
            /* quadratic form of the polynomial smoothness indicator */
            for (int i = 0; i <= R; ++i)
                for (int j = 0; j <= R; ++j) b += B[16 * m + 4 * i + j] * fm[i] * fm[j];
        } else {
            /* zero mean: the data itself; non-zero mean: its deviation from the
             * centre cell's value f[R] */
            double mean = nonzero_mean ? f[R] : 0.0;
            for (int i = 0; i <= R; ++i) {
                double proj = 0.0;
                for (int j = 0; j <= R; ++j) proj += P[4 * i + j] * (fm[j] - mean);
                b += proj * proj;
            }
        }
        beta[m] = b;
        double a = 0.0, z = 0.0;
        for (int j = 0; j <= R; ++j) {
            a += wp[4 * m + j] * fm[j];
            z += wm[4 * m + j] * fm[j];
        }
        qp[m] = a;
        qm[m] = z;
        double den = (EPS_WENO + b) * (EPS_WENO + b);
        wtp[m] = gp[m] / den;
        wtm[m] = gm[m] / den;
        sp += wtp[m];
        sm += wtm[m];
    }
    double accp = 0.0, accm = 0.0;
    for (int m = 0; m <= R; ++m) {
        double op = wtp[m] / sp, om = wtm[m] / sm;
        accp += op * qp[m];
        accm += om * qm[m];
        if (beta_out) beta_out[m] = beta[m];
        if (omp_out) omp_out[m] = op;
        if (omm_out) omm_out[m] = om;
    }
    *qplus = accp;
    *qminus = accm;
}

/* ---------------------------------------------------------------------------
 * HLLC approximate Riemann solver (Sec. 7 intro names HLLC; textbook form),
 * left/right primitive states in the rotated frame, flux in the rotated frame.
 * ------------------------------------------------------------------------- */
void oracle_hllc(const double *qL, const double *qR, double gamma, double *F) {
    double FL[5], FR[5], UL[5], UR[5];
    phys_flux(qL, gamma, FL, UL);
    phys_flux(qR, gamma, FR, UR);
    double rL = qL[Q_RHO], uL = qL[Q_UN], pL = qL[Q_P];
    double rR = qR[Q_RHO], uR = qR[Q_UN], pR = qR[Q_P];
    double cL = sqrt(gamma * pL / rL), cR = sqrt(gamma * pR / rR);
    double SL = fmin(uL - cL, uR - cR);
    double SR = fmax(uL + cL, uR + cR);
    double Sstar = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
                   (rL * (SL - uL) - rR * (SR - uR));
    if (SL >= 0.0) {
        for (int k = 0; k < 5; ++k) F[k] = FL[k];
        return;
    }
    if (SR <= 0.0) {
        for (int k = 0; k < 5; ++k) F[k] = FR[k];
        return;
    }
    const double *q = (Sstar >= 0.0) ? qL : qR;
    const double *Fk = (Sstar >= 0.0) ? FL : FR;
    const double *Uk = (Sstar >= 0.0) ? UL : UR;
    double S = (Sstar >= 0.0) ? SL : SR;
    double rho = q[Q_RHO], un = q[Q_UN], p = q[Q_P];
    double fac = rho * (S - un) / (S - Sstar);
    double Us[5];
    Us[0] = fac;
    Us[1] = fac * Sstar;
    Us[2] = fac * q[Q_UT1];
    Us[3] = fac * q[Q_UT2];
    Us[4] = fac * (Uk[4] / rho + (Sstar - un) * (Sstar + p / (rho * (S - un))));
    for (int k = 0; k < 5; ++k) F[k] = Fk[k] + S * (Us[k] - Uk[k]);
}

/* Corrected numerical flux at face j+1/2 from the face fluxes F_{j-3/2} .. F_{j+5/2}
 * (Eqs. (numFlux_cor), (FD-ders)); the dx^2 and dx^4 factors cancel. */
double oracle_flux_hat(const double *F5) {
    double d2 = F5[1] - 2.0 * F5[2] + F5[3];
    double d4 = F5[0] - 4.0 * F5[1] + 6.0 * F5[2] - 4.0 * F5[3] + F5[4];
    return F5[2] + ALPHA_FC * d2 + BETA_FC * d4;
}

/* The same with the sixth-difference term, from F_{j-5/2} .. F_{j+7/2}. */
double oracle_flux_hat7(const double *F7) {
    double d2 = F7[2] - 2.0 * F7[3] + F7[4];
    double d4 = F7[1] - 4.0 * F7[2] + 6.0 * F7[3] - 4.0 * F7[4] + F7[5];
    double d6 = F7[0] - 6.0 * F7[1] + 15.0 * F7[2] - 20.0 * F7[3] + 15.0 * F7[4] - 6.0 * F7[5] + F7[6];
    return F7[3] + ALPHA_FC * d2 + BETA_FC * d4 + C6_FC * d6;
}

/* Terms of the correction in use (2 or 3). */
static int corr_terms(const oracle_cfg *c) { return c->flux_corr_terms == 3 ? 3 : 2; }

/* Reconstruct the Riemann states of one cell: the 2R+1 rotated primitive
 * vectors qs[0..2R] (centre at index R) -> q^+ at x_{i+1/2}, q^- at x_{i-1/2}. */
static int reconstruct_cell(const oracle_cfg *c, int d, const double (*qs)[5],
                            double *qplus, double *qminus) {
    int R = c->R;
    int kf[5];
    int nk = active_fields(c->ndim, kf);
    double L[5][5], Rv[5][5];
    oracle_char_vectors(qs[R], c->gamma, &L[0][0], &Rv[0][0]);
    double Wp[5] = {0, 0, 0, 0, 0}, Wm[5] = {0, 0, 0, 0, 0};
    for (int a = 0; a < nk; ++a) {
        int k = kf[a];
        double f[2 * RMAX + 1];
        for (int s = 0; s <= 2 * R; ++s) {
            double w = 0.0;
            for (int q = 0; q < 5; ++q) w += L[k][q] * qs[s][q];
            f[s] = w;
        }
        if (c->ao) {
            for (int side = 0; side < 2; ++side)
                oracle_gp_ao(R, f, c->ao_w7[d][side], c->ao_w5[d][side], &c->ao_w3[d][side][0][0],
                             &c->ao_P7[d][0][0], &c->ao_P5[d][0][0], &c->ao_P3[d][0][0], c->ao_c[d],
                             c->ao_gam, side == 0 ? &Wp[k] : &Wm[k], NULL);
        } else {
            oracle_gp_weno(R, f, &c->wp[d][0][0], &c->wm[d][0][0], c->gp[d], c->gm[d],
                           &c->P[d][0][0], c->beta_form ? &c->B[d][0][0][0] : NULL, c->nonzero_mean,
                           &Wp[k], &Wm[k], NULL, NULL, NULL);
        }
    }
    for (int q = 0; q < 5; ++q) {
        double ap = 0.0, am = 0.0;
        for (int a = 0; a < nk; ++a) {
            int k = kf[a];
            ap += Wp[k] * Rv[k][q];
            am += Wm[k] * Rv[k][q];
        }
        qplus[q] = ap;
        qminus[q] = am;
    }
    int fallbacks = 0;
    if (c->positivity_fallback) {
        if (!(qplus[Q_RHO] > 0.0) || !(qplus[Q_P] > 0.0)) {
            for (int q = 0; q < 5; ++q) qplus[q] = qs[R][q];
            ++fallbacks;
        }
        if (!(qminus[Q_RHO] > 0.0) || !(qminus[Q_P] > 0.0)) {
            for (int q = 0; q < 5; ++q) qminus[q] = qs[R][q];
            ++fallbacks;
        }
    }
    return fallbacks;
}

/* ---------------------------------------------------------------------------
 * Right-hand side of Eq. (disc_fd): Lout = -sum_d (fhat_{+1/2} - fhat_{-1/2})/dx_d.
 * Directions are processed x, y, z; each pencil along d is independent.
 * Returns the number of positivity fallbacks taken.
 * ------------------------------------------------------------------------- */
long oracle_rhs(const oracle_cfg *c, const double *U, double *Lout) {
    int ndim = c->ndim, nv = 2 + ndim, R = c->R;
    size_t ncell = ncells_of(c);
    double *Vp = (double *)malloc(sizeof(double) * 5 * ncell);
    for (size_t i = 0; i < ncell; ++i) {
        double u[NVMAX], v5[5];
        for (int k = 0; k < nv; ++k) u[k] = U[(size_t)k * ncell + i];
        oracle_cons_to_prim(ndim, c->gamma, u, v5);
        for (int k = 0; k < 5; ++k) Vp[(size_t)k * ncell + i] = v5[k];
    }
    memset(Lout, 0, sizeof(double) * nv * ncell);
    long fallbacks = 0;
    for (int d = 0; d < ndim; ++d) {
        int N = c->n[d];
        size_t stride = 1;
        for (int e = 0; e < d; ++e) stride *= (size_t)c->n[e];
        size_t npencil = ncell / (size_t)N;
        int ax[3];
        frame_axes(d, ax);
        /* conserved-momentum slot for each rotated component */
        int slot[5] = {0, 1 + ax[0], 1 + ax[1], 1 + ax[2], nv - 1};
        /* ghost cells: the stencil radius, the nc face fluxes either side of a
         * face that the correction takes, and the face of the difference */
        int nc = corr_terms(c);
        int G = R + 1 + nc;
        double inv_dx = 1.0 / c->dx[d];
#pragma omp parallel for schedule(static) reduction(+ : fallbacks)
        for (long pi = 0; pi < (long)npencil; ++pi) {
            /* base offset of the pencil: decompose pi over the other axes */
            size_t lo = (size_t)pi % stride, hi = (size_t)pi / stride;
            size_t base = lo + hi * stride * (size_t)N;
            int len = N + 2 * G;
            double (*q)[5] = malloc(sizeof(double) * 5 * len);
            double (*qplus)[5] = malloc(sizeof(double) * 5 * len);
            double (*qminus)[5] = malloc(sizeof(double) * 5 * len);
            double (*Ff)[5] = malloc(sizeof(double) * 5 * len);
            double *fh = malloc(sizeof(double) * 5 * len);
            /* gather the pencil with G ghost cells per side, rotated to direction d.
             * Ghosts: periodic images; outflow copies the boundary cell
             * (zero gradient); a reflecting wall mirrors the cells about the
             * boundary face with the normal velocity reversed. */
            for (int s = 0; s < len; ++s) {
                int i = s - G, flip = 0;
                if (i < 0 || i >= N) {
                    int kind = c->bc[d][i < 0 ? 0 : 1];
                    if (kind == BC_PERIODIC) {
                        i = ((i % N) + N) % N;
                    } else if (kind == BC_OUTFLOW) {
                        i = i < 0 ? 0 : N - 1;
                    } else {
                        i = i < 0 ? -1 - i : 2 * N - 1 - i;
                        flip = 1;
                    }
                }
                size_t cell = base + (size_t)i * stride;
                q[s][Q_RHO] = Vp[0 * ncell + cell];
                q[s][Q_UN] = (flip ? -1.0 : 1.0) * Vp[(size_t)(1 + ax[0]) * ncell + cell];
                q[s][Q_UT1] = Vp[(size_t)(1 + ax[1]) * ncell + cell];
                q[s][Q_UT2] = Vp[(size_t)(1 + ax[2]) * ncell + cell];
                q[s][Q_P] = Vp[(size_t)4 * ncell + cell];
            }
            /* Riemann states of cells -(nc+1) .. N+nc (pencil index s = i + G) */
            for (int i = -(nc + 1); i <= N + nc; ++i) {
                int s = i + G;
                fallbacks += reconstruct_cell(c, d, (const double (*)[5])&q[s - R], qplus[s], qminus[s]);
            }
            /* face fluxes F_{j+1/2}, j = -(nc+1) .. N+nc-1 (Eq. (riemann_prob)) */
            for (int j = -(nc + 1); j <= N + nc - 1; ++j) {
                int s = j + G;
                oracle_hllc(qplus[s], qminus[s + 1], c->gamma, Ff[s]);
            }
            /* corrected fluxes fhat_{j+1/2}, j = -1 .. N-1, and the update */
            for (int j = -1; j <= N - 1; ++j) {
                int s = j + G;
                for (int k = 0; k < 5; ++k) {
                    double Fn[7];
                    for (int o = -nc; o <= nc; ++o) Fn[o + nc] = Ff[s + o][k];
                    fh[5 * s + k] = nc == 3 ? oracle_flux_hat7(Fn) : oracle_flux_hat(Fn);
                }
            }
            for (int i = 0; i < N; ++i) {
                int s = i + G;
                size_t cell = base + (size_t)i * stride;
                for (int k = 0; k < 5; ++k) {
                    int sl = slot[k];
                    if (k == Q_UT1 && ndim < 2) continue;
                    if (k == Q_UT2 && ndim < 3) continue;
                    Lout[(size_t)sl * ncell + cell] += -(fh[5 * s + k] - fh[5 * (s - 1) + k]) * inv_dx;
                }
            }
            free(q); free(qplus); free(qminus); free(Ff); free(fh);
        }
    }
    free(Vp);
    return fallbacks;
}

/* Largest sum_d (|u_d| + c)/dx_d over all cells (the CFL reading). */
double oracle_max_speed(const oracle_cfg *c, const double *U) {
    int ndim = c->ndim, nv = 2 + ndim;
    size_t ncell = ncells_of(c);
    double smax = 0.0;
    for (size_t i = 0; i < ncell; ++i) {
        double u[NVMAX], v5[5];
        for (int k = 0; k < nv; ++k) u[k] = U[(size_t)k * ncell + i];
        oracle_cons_to_prim(ndim, c->gamma, u, v5);
        double cs = sqrt(c->gamma * v5[4] / v5[0]);
        double s = 0.0;
        for (int d = 0; d < ndim; ++d) s += (fabs(v5[1 + d]) + cs) / c->dx[d];
        if (s > smax || s != s) smax = s;
    }
    return smax;
}

/* One SSP-RK3 stage in Shu-Osher form (Sec. 7 intro: third-order TVD RK):
 *   stage 1: out = Uin + dt L
 *   stage 2: out = 3/4 Un + 1/4 (Uin + dt L)
 *   stage 3: out = 1/3 Un + 2/3 (Uin + dt L)                                  */
void oracle_rk3_combine(int stage, size_t count, const double *Un, const double *Uin,
                        const double *L, double dt, double *out) {
    for (size_t i = 0; i < count; ++i) {
        double adv = Uin[i] + dt * L[i];
        if (stage == 1) out[i] = adv;
        else if (stage == 2) out[i] = 0.75 * Un[i] + 0.25 * adv;
        else out[i] = (1.0 / 3.0) * Un[i] + (2.0 / 3.0) * adv;
    }
}

/* One full SSP-RK3 step with a given dt. U is updated in place. */
long oracle_step_dt(const oracle_cfg *c, double *U, double dt) {
    size_t count = (size_t)(2 + c->ndim) * ncells_of(c);
    double *U1 = malloc(sizeof(double) * count);
    double *U2 = malloc(sizeof(double) * count);
    double *L = malloc(sizeof(double) * count);
    long fb = 0;
    fb += oracle_rhs(c, U, L);
    oracle_rk3_combine(1, count, U, U, L, dt, U1);
    fb += oracle_rhs(c, U1, L);
    oracle_rk3_combine(2, count, U, U1, L, dt, U2);
    fb += oracle_rhs(c, U2, L);
    oracle_rk3_combine(3, count, U, U2, L, dt, U);
    free(U1); free(U2); free(L);
    return fb;
}

/* CFL time step from the current state, clipped to t_final. */
double oracle_dt(const oracle_cfg *c, const double *U, double cfl, double t, double t_final) {
    double dt = cfl / oracle_max_speed(c, U);
    if (t + dt > t_final) dt = t_final - t;
    return dt;
}

/* Advance to t_final (or at most max_steps steps) with the CFL time step.
 * Returns the number of positivity fallbacks; *t and *nsteps are updated. */
long oracle_run(const oracle_cfg *c, double *U, double cfl, double t_final, long max_steps,
                double *t, long *nsteps) {
    long fb = 0;
    while (*t < t_final && (max_steps < 0 || *nsteps < max_steps)) {
        double dt = oracle_dt(c, U, cfl, *t, t_final);
        fb += oracle_step_dt(c, U, dt);
        *t += dt;
        *nsteps += 1;
    }
    return fb;
}

/* Advance exactly nsteps steps of a fixed dt (convergence studies). */
long oracle_run_fixed(const oracle_cfg *c, double *U, double dt, long nsteps) {
    long fb = 0;
    for (long s = 0; s < nsteps; ++s) fb += oracle_step_dt(c, U, dt);
    return fb;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Size of oracle_cfg, so the loader can check its mirror of the struct. */
size_t oracle_cfg_size(void) { return sizeof(oracle_cfg); }
