// GP-WENO FD-Prim sweep kernels for gfx950 (CDNA4, wave64).
//
// One kernel launch evaluates one direction's contribution to the right-hand
// side of Eq. (disc_fd) for every cell. The sweeps of an RK stage run z, y, x,
// and the x sweep also finishes the stage. Work decomposition:
//
//   * A "run" is 64 consecutive cells of one pencil along the sweep axis,
//     mapped one cell per lane of a wave. Each lane reconstructs the Riemann
//     states of its cell (stencil of 2R+1 cells read from LDS), the wave then
//     forms face fluxes, corrected fluxes and flux differences exchanging
//     neighbouring lanes' values with DPP wave shifts. The flux correction
//     needs face fluxes NC faces either side (NC = 2: alpha and beta; 3: also
//     the sixth difference) and the difference one more face, so lanes
//     NC+1 .. 62-NC produce output: a run yields 58 cells (56 with NC = 3),
//     and consecutive runs overlap by 6 (8) cells.
//   * A block holds several pencils (one wave each) and the same run segment.
//     The input tile [2+ndim fields][pencils][64 + 2R cells] is loaded once
//     from HBM (ghost positions: periodic image, outflow copy or mirror image),
//     converted to rotated primitive variables and staged in LDS.
//   * x sweeps: each wave loads its own row (contiguous along x) and writes its
//     outputs directly (contiguous). y/z sweeps: a block holds 4 adjacent
//     x-columns (8 for float32 3D grids, see sweep_wpb), so every global access
//     covers 4 (8) consecutive doubles; the outputs are transposed through LDS
//     so the accumulator's read-modify-write is also x-contiguous.
//
// Per cell (paper references):
//   characteristic projection of the primitive stencil at the centre cell
//     (Sec. 7 intro), GP-WENO per field (Sec. 3.3: Eqs. (candidate_interp),
//     (beta-eigen), (weights), (weight_sum)), back-projection, HLLC at the face
//     (Eq. (riemann_prob)), flux correction alpha = -1/24, beta = 3/640
//     (Eqs. (numFlux_cor), (FD-ders)), flux difference (Eq. (disc_fd)), SSP-RK3.
//
// Precision: Real is the sweep arithmetic type (double or float). The state,
// flux differences, accumulator, RK combination, CFL speeds and sums are
// always float64; a float32 corrected flux is widened before its difference
// is taken, so both neighbours of a face subtract the same value.
#include <float.h>
#include <limits.h>

#pragma once

#include "gpweno_kernels.h"

namespace gpw {


// Pencils (waves) per block: 4 rows in x sweeps, 4 adjacent x columns in y/z
// sweeps. Four-wave blocks fill the register-limited wave slots of a compute
// unit without stranding any, and spread small grids evenly over the compute
// units (eight-wave y blocks left a 512^2 grid at 2.25 blocks per unit).
// float32 y/z sweeps of 3D grids take 8 columns: their tile rows become 64
// contiguous bytes of float64 state instead of 32, which shortens those sweeps
// by 5-10 % on a 256^3 grid; float64 ones, at four waves per SIMD, lose as much.
__host__ __device__ constexpr int sweep_wpb(int ndim, int dir, bool fp32) {
    return (ndim == 3 && dir != 0 && fp32) ? 8 : 4;
}

__host__ __device__ constexpr int t1_axis(int dir) { return dir == 0 ? 1 : 0; }
__host__ __device__ constexpr int t2_axis(int dir) { return dir == 2 ? 1 : 2; }

// Conserved slot of rotated component k (rho, u_n, u_t1, u_t2, p order).
template <int NDIM, int DIR>
__host__ __device__ constexpr int cons_slot(int k) {
    return k == 0 ? 0
         : k == 1 ? 1 + DIR
         : k == 1 + NDIM ? 1 + NDIM
         : k == 2 ? 1 + t1_axis(DIR)
         : 1 + t2_axis(DIR);
}

// Reciprocal and reciprocal square root. float: the hardware approximations
// (about 1 ulp). double: the hardware approximation refined by two Newton-Raphson
// steps, r <- r + r (1 - x r) and y <- y + y (1 - x y^2)/2, each of which squares
// the relative error, giving float64 accuracy to within an ulp or two; cheaper
// than the IEEE division and square-root sequences. Arguments are positive and
// normal wherever these are used on a selected value.
template <typename Real> __device__ __forceinline__ Real frcp(Real x);
template <> __device__ __forceinline__ float frcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double frcp<double>(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
template <typename Real> __device__ __forceinline__ Real frsq(Real x);
template <> __device__ __forceinline__ float frsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double frsq<double>(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// Value of the neighbouring lane across the whole wave, by DPP wave shifts
// (wave_shr:1 / wave_shl:1): lane_prev gives lane l the value of lane l-1,
// lane_next the value of lane l+1; the lane without a neighbour gets 0 (its
// result is never used: a run's outputs come from lanes NC+1 .. 62-NC). One VALU move,
// which the compiler can fold into the consuming instruction, instead of a
// permute through the LDS crossbar.
__device__ __forceinline__ float lane_prev(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_next(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ double lane_prev(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_next(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Periodic index. For n >= 64 every index a sweep forms lies in [-n, 2n), so a
// compare-and-add suffices; shorter axes (tests) take the general modulo.
__device__ __forceinline__ int wrap(int x, int n) {
    if (n >= WAVE) {
        x += (x < 0) ? n : 0;
        return x - ((x >= n) ? n : 0);
    }
    int r = x % n;
    return r < 0 ? r + n : r;
}

// Source cell of stencil position x on an axis of n cells, for the boundary kinds
// lo / hi of its two sides (gpweno_bc: 0 periodic, 1 outflow, 2 reflecting), and
// whether the normal momentum changes sign (mirror image at a wall). Positions
// beyond the ghost depth (unused lanes of a pencil's last run) are clamped into
// the axis so every load stays in bounds.
__device__ __forceinline__ int ghost_src(int x, int n, int lo, int hi, bool& flip) {
    flip = false;
    if (x >= 0 && x < n) return x;
    const int kind = x < 0 ? lo : hi;
    if (kind == 0) return wrap(x, n);
    int j;
    if (kind == 1) {
        j = x < 0 ? 0 : n - 1;
    } else {
        j = x < 0 ? -1 - x : 2 * n - 1 - x;
        flip = true;
    }
    return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// dt of step n starting at t0 from the CFL speeds of its initial state (the
// max over the per-XCD slots n & 1), or the fixed step, clipped to t_final.
__device__ __forceinline__ double step_dt(const Ctl* c, long long n, double t0) {
    unsigned long long smax = 0;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const unsigned long long v = c->xcd[x].speed[n & 1];
        smax = v > smax ? v : smax;
    }
    const double speed = __longlong_as_double((long long)smax);
    double d = c->fixed_dt > 0.0 ? c->fixed_dt : c->cfl / speed;
    if (t0 + d > c->t_final) d = c->t_final - t0;
    return d;
}

// Time step of the step in flight and whether it runs. final_sweep: the
// sweep that closes the step (its block 0 writes the next step state). Only
// sweeps that finish an RK stage need dt (NEED_DT): from the value the step's
// first sweep stored, or, for a first sweep that finishes a stage itself
// (from_speeds, 1D only), from the CFL speeds. The fields are read up front,
// with no address depending on another read, so the control block costs one
// round trip of scalar loads; the speeds of the from_speeds path follow once
// the step count is known.
template <bool NEED_DT>
__device__ __forceinline__ bool step_go(const Ctl* c, bool final_sweep, bool from_speeds, double& t0, double& dt,
                                        long long& n) {
    const long long n0 = c->rec[0].nsteps, n1 = c->rec[1].nsteps;
    const double ta = c->rec[0].t, tb = c->rec[1].t;
    const long long st = c->started;
    const int err = c->err;
    const double tf = c->t_final;
    const long long lim = c->step_limit;
    double d0 = 0.0, d1 = 0.0;
    if (NEED_DT && !from_speeds) {
        d0 = c->dt_step[0];
        d1 = c->dt_step[1];
    }
    int r;
    if (final_sweep) {
        if (st < 0) return false;
        r = (n0 == st) ? 0 : 1;
        if ((r ? n1 : n0) != st) return false;
    } else {
        r = n0 > n1 ? 0 : 1;
    }
    t0 = r ? tb : ta;
    n = r ? n1 : n0;
    if (err || !(t0 < tf) || n >= lim) return false;
    if (NEED_DT) dt = from_speeds ? step_dt(c, n, t0) : ((n & 1) ? d1 : d0);
    return true;
}

// Conserved -> primitive in the frame rotated to DIR: (rho, u_n[, u_t1[, u_t2]], p).
template <int NDIM, int DIR>
__device__ __forceinline__ void cons_to_rot(const double (&u)[2 + NDIM], double gamma, double q[2 + NDIM]) {
    constexpr int NV = 2 + NDIM;
    const double rho = u[0];
    const double irho = frcp(rho);
    double vel[3] = {0.0, 0.0, 0.0};
    double ke = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        vel[d] = u[1 + d] * irho;
        ke += vel[d] * u[1 + d];
    }
    const double E = u[NV - 1];
    q[0] = rho;
    q[1] = vel[DIR];
    if (NDIM >= 2) q[2] = vel[t1_axis(DIR)];
    if (NDIM == 3) q[3] = vel[t2_axis(DIR)];
    q[NV - 1] = (gamma - 1.0) * (E - 0.5 * ke);
}

// GP-WENO interpolation of one characteristic field f[0..2R] to x_{i+1/2} (qp)
// and x_{i-1/2} (qm). beta_m = sum_i (P_m,i . f_m)^2 is shared by both points.
// The comparison schemes (polynomial WENO with Jiang-Shu or GP smoothness
// indicators) run through the same code with their own tables. IK, the kind of
// smoothness indicator:
//   0  GP, zero mean: the one factor of K_m(sigma), the same for every m, read
//      once (fewer scalar registers for the tables);
//   1  a factor per sub-stencil of rank R (Jiang-Shu quadratic forms);
//   2  GP with the centre cell's value as the mean: the factor of K_m(sigma)
//      applied to f_m - f_i (the paper's non-zero-mean variant, Sec. 7).
// Nonlinear weights gamma_m / (eps + beta_m)^2 are evaluated, in float32, in
// the equivalent form gamma_m * ((eps + beta_min)/(eps + beta_m))^2, which
// cannot overflow or underflow to 0/0 (eps = 1e-36 squared is below float
// range), and in float64 over a common denominator, without reciprocals.
// The weights of x_{i-1/2} are those of x_{i+1/2} mirrored about the centre
// cell (the covariance kernel and the stencils are symmetric): sub-stencil m,
// node j at -1/2 takes w_{R-m, R-j} at +1/2 and gamma_m takes gamma_{R-m}.
// Reading one set halves the tables a sweep holds in scalar registers.
template <int R, typename Real, int IK>
__device__ __forceinline__ void gp_weno(const Real (&f)[2 * R + 1], const Tab<Real>& T, Real& qp, Real& qm) {
    Real e[R + 1], cp[R + 1], cm[R + 1];
    Real g[2 * R + 1];  // the data the indicators see
#pragma unroll
    for (int j = 0; j <= 2 * R; ++j) g[j] = IK == 2 ? f[j] - f[R] : f[j];
#pragma unroll
    for (int m = 0; m <= R; ++m) {
        // e_m = eps + beta_m, with eps = 1e-36 as the start of the accumulation
        Real b;
        if constexpr (IK != 1 && R >= 2) {
            // GP rows in symmetric / antisymmetric form: K(sigma) is symmetric
            // Toeplitz, so every eigenvector is symmetric or antisymmetric about
            // the sub-stencil centre, and acts on mirrored sums or differences
            // (10 instead of 12 operations for R = 2, 16 instead of 20 for R = 3)
            const Real s0 = g[m] + g[m + R], d0 = g[m] - g[m + R];
            const Real s1 = R == 2 ? g[m + 1] : g[m + 1] + g[m + 2];
            const Real p0 = fma(T.Ps[0][0], s0, T.Ps[0][1] * s1);
            const Real p1 = fma(T.Ps[1][0], s0, T.Ps[1][1] * s1);
            if constexpr (R == 2) {
                const Real p2 = T.Ps[2][0] * d0;
                b = fma(p0, p0, fma(p1, p1, fma(p2, p2, Real(1e-36))));
            } else {
                const Real d1 = g[m + 1] - g[m + 2];
                const Real p2 = fma(T.Ps[2][0], d0, T.Ps[2][1] * d1);
                const Real p3 = fma(T.Ps[3][0], d0, T.Ps[3][1] * d1);
                b = fma(p0, p0, fma(p1, p1, fma(p2, p2, fma(p3, p3, Real(1e-36)))));
            }
        } else {
            b = Real(1e-36);
#pragma unroll
            for (int i = 0; i < (IK == 1 ? R : R + 1); ++i) {  // Jiang-Shu forms have rank R
                Real pr = T.P[IK == 1 ? m : 0][i][0] * g[m];
#pragma unroll
                for (int j = 1; j <= R; ++j) pr = fma(T.P[IK == 1 ? m : 0][i][j], g[m + j], pr);
                b = fma(pr, pr, b);
            }
        }
        e[m] = b;
        // gamma_m q_m at both points (the candidates enter only in that product)
        Real ap = T.gwp[m][0] * f[m];
        Real am = T.gwp[R - m][R] * f[m];
#pragma unroll
        for (int j = 1; j <= R; ++j) {
            ap = fma(T.gwp[m][j], f[m + j], ap);
            am = fma(T.gwp[R - m][R - j], f[m + j], am);
        }
        cp[m] = ap;
        cm[m] = am;
    }
    // w_m: 1/e_m^2 up to a factor common to all m
    Real w[R + 1];
    if constexpr (sizeof(Real) == 8) {
        // float64: over the common denominator prod_k e_k^2, w_m = prod_{k != m}
        // e_k^2, with no reciprocal. From e_k >= eps = 1e-36 up to 1e51 (R = 3)
        // or 1e77 (R <= 2) every product below and the sums sp, sm stay normal
        // doubles; beyond that (GP data of magnitude about 1e24 for R = 3, 1e37
        // for R <= 2) they overflow, the interpolant becomes NaN and the stage
        // check reports a non-physical state.
        Real E[R + 1];
#pragma unroll
        for (int m = 0; m <= R; ++m) E[m] = e[m] * e[m];
        if constexpr (R == 1) {
            w[0] = E[1];
            w[1] = E[0];
        } else if constexpr (R == 2) {
            w[0] = E[1] * E[2];
            w[1] = E[0] * E[2];
            w[2] = E[0] * E[1];
        } else {
            const Real e01 = E[0] * E[1], e23 = E[2] * E[3];
            w[0] = E[1] * e23;
            w[1] = E[0] * e23;
            w[2] = e01 * E[3];
            w[3] = e01 * E[2];
        }
    } else {
        // float32: as ratios to the smallest e_m, (e_min / e_m)^2 in (0, 1]
        Real emin = e[0];
#pragma unroll
        for (int m = 1; m <= R; ++m) emin = fmin(emin, e[m]);
#pragma unroll
        for (int m = 0; m <= R; ++m) {
            const Real r = emin * frcp(e[m]);
            w[m] = r * r;
        }
    }
    // q = sum_m w_m gamma_m q_m / sum_m w_m gamma_m at each point
    Real sp = T.gp[0] * w[0], sm = T.gp[R] * w[0], accp = w[0] * cp[0], accm = w[0] * cm[0];
#pragma unroll
    for (int m = 1; m <= R; ++m) {
        sp = fma(T.gp[m], w[m], sp);
        sm = fma(T.gp[R - m], w[m], sm);
        accp = fma(w[m], cp[m], accp);
        accm = fma(w[m], cm[m], accm);
    }
    if constexpr (sizeof(Real) == 8) {
        // sp sm would leave the double range: normalised one at a time
        qp = accp * frcp(sp);
        qm = accm * frcp(sm);
    } else {
        // both normalisations from one reciprocal: 1/sp = sm/(sp sm), 1/sm = sp/(sp sm)
        const Real inv = frcp(sp * sm);
        qp = accp * (sm * inv);
        qm = accm * (sp * inv);
    }
}

// Adaptive-order GP interpolation (the paper's App. A) of one characteristic
// field f[0..2R] to x_{i+1/2} (qp) and x_{i-1/2} (qm); R = 3 gives GP-AO(3,2,3),
// R = 2 gives GP-AO(2,3).
//   indicators: the negative log-likelihood with its normalisation and
//     complexity terms, beta_N = c_N + 1/2 sum_i (P_i . f_N)^2 (Eqs. (log-like),
//     (beta-eigen)), for the 7- and 5-point stencils and the three 3-point
//     sub-stencils of the 5-point one;
//   GP-AO(R,3): omega^R and omega_m from gamma_HI/(eps+beta^R)^2 and
//     gamma_m/(eps+beta_m)^2 normalised together (Eq. (nonlin-AO), with gamma_m
//     for the sub-stencils), q = omega^R/gamma_HI q^R + sum_m (omega_m -
//     omega^R gamma_m/gamma_HI) q^m (Eq. (GP-AO));
//   GP-AO(3,2,3): weights gamma_HI/(eps+beta^7)^2 and (1-gamma_HI)/(eps+beta^5)^2
//     normalised (Eq. (recursive-weights)) combine the two (Eq. (AO-recursive)).
// The weights are evaluated as ratios to the smallest |eps + beta| (the
// indicators can be negative: the log-det term of a 7-point K is), so no
// intermediate overflows. Both faces share the indicators and weights; the
// interpolation weights of x_{i-1/2} are those of x_{i+1/2} mirrored.
template <int N, typename Real>
__device__ __forceinline__ Real half_quad(const Real (&P)[N][N], const Real* f) {
    Real s = Real(0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        Real pr = P[i][0] * f[0];
#pragma unroll
        for (int j = 1; j < N; ++j) pr = fma(P[i][j], f[j], pr);
        s = fma(pr, pr, s);
    }
    return Real(0.5) * s;
}

// Coefficients (a_hi, a_m) of q = a_hi q^hi + sum_m a_m q^m for GP-AO(R,3)
// given e = eps + beta of the high-order stencil and of the sub-stencils.
template <typename Real>
__device__ __forceinline__ void ao_coeffs(Real eh, const Real (&em)[3], const Tab<Real>& T, Real& ah, Real (&am)[3]) {
    Real mn = fabs(eh);
#pragma unroll
    for (int m = 0; m < 3; ++m) mn = fmin(mn, fabs(em[m]));
    const Real ghi = T.ao.ghi;
    Real r = mn * frcp(eh);
    const Real wh = ghi * r * r;
    Real wm[3], sum = wh;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        r = mn * frcp(em[m]);
        wm[m] = T.gp[m] * r * r;
        sum += wm[m];
    }
    const Real inv = frcp(sum);
    ah = wh * inv * frcp(ghi);
#pragma unroll
    for (int m = 0; m < 3; ++m) am[m] = fma(-ah, T.gp[m], wm[m] * inv);
}

template <int R, typename Real>
__device__ __forceinline__ void gp_ao(const Real (&f)[2 * R + 1], const Tab<Real>& T, Real& qp, Real& qm) {
    static_assert(R == 2 || R == 3, "GP-AO uses stencils of radius 2 and 3");
    const Real* f5 = f + (R - 2);
    const Real e5 = Real(1e-36) + (T.ao.c[1] + half_quad<5, Real>(T.ao.P5, f5));
    Real em[3], q3p[3], q3m[3];
    Real P3[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) P3[i][j] = T.P[0][i][j];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        em[m] = Real(1e-36) + (T.ao.c[2] + half_quad<3, Real>(P3, f5 + m));
        Real a = T.wp[m][0] * f5[m], b = T.wp[2 - m][2] * f5[m];
#pragma unroll
        for (int j = 1; j < 3; ++j) {
            a = fma(T.wp[m][j], f5[m + j], a);
            b = fma(T.wp[2 - m][2 - j], f5[m + j], b);
        }
        q3p[m] = a;
        q3m[m] = b;
    }
    Real q5p = T.ao.w5p[0] * f5[0], q5m = T.ao.w5p[4] * f5[0];
#pragma unroll
    for (int j = 1; j < 5; ++j) {
        q5p = fma(T.ao.w5p[j], f5[j], q5p);
        q5m = fma(T.ao.w5p[4 - j], f5[j], q5m);
    }
    Real a5, c5[3];
    ao_coeffs<Real>(e5, em, T, a5, c5);
    Real ao5p = a5 * q5p, ao5m = a5 * q5m;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        ao5p = fma(c5[m], q3p[m], ao5p);
        ao5m = fma(c5[m], q3m[m], ao5m);
    }
    if constexpr (R == 2) {
        qp = ao5p;
        qm = ao5m;
    } else {
        const Real e7 = Real(1e-36) + (T.ao.c[0] + half_quad<7, Real>(T.ao.P7, f));
        Real q7p = T.ao.w7p[0] * f[0], q7m = T.ao.w7p[6] * f[0];
#pragma unroll
        for (int j = 1; j < 7; ++j) {
            q7p = fma(T.ao.w7p[j], f[j], q7p);
            q7m = fma(T.ao.w7p[6 - j], f[j], q7m);
        }
        Real a7, c7[3];
        ao_coeffs<Real>(e7, em, T, a7, c7);
        Real ao7p = a7 * q7p, ao7m = a7 * q7m;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            ao7p = fma(c7[m], q3p[m], ao7p);
            ao7m = fma(c7[m], q3m[m], ao7m);
        }
        // recursive weights of the 7- and 5-point stencils, as ratios
        const Real ghi = T.ao.ghi;
        const Real mn = fmin(fabs(e7), fabs(e5));
        Real r = mn * frcp(e7);
        const Real nh = ghi * r * r;
        r = mn * frcp(e5);
        const Real nl = (Real(1) - ghi) * r * r;
        const Real inv = frcp(nh + nl);
        const Real bh = nh * inv * frcp(ghi);
        const Real bl = fma(-bh, Real(1) - ghi, nl * inv);
        qp = fma(bh, ao7p, bl * ao5p);
        qm = fma(bh, ao7m, bl * ao5m);
    }
}

// The interpolation of one field for the indicator kind.
template <int R, typename Real, int IK>
__device__ __forceinline__ void interp(const Real (&f)[2 * R + 1], const Tab<Real>& T, Real& qp, Real& qm) {
    if constexpr (IK == 3) gp_ao<R, Real>(f, T, qp, qm);
    else gp_weno<R, Real, IK>(f, T, qp, qm);
}

// Riemann states of the cell at lane position l: stencil entries l .. l+2R of a
// pencil in LDS (field k at s[k * fs + .]). Projects the primitive stencil on the
// left eigenvectors of the primitive Jacobian at the centre cell, interpolates
// each characteristic field, and projects back with the right eigenvectors:
//   acoustic -:  -rho/(2c) u_n + p/(2c^2)       r = (1, -c/rho, 0, 0, c^2)
//   entropy   :  rho - p/c^2                    r = (1, 0, 0, 0, 0)
//   shear     :  u_t1, u_t2                     r = unit vectors
//   acoustic +:   rho/(2c) u_n + p/(2c^2)       r = (1,  c/rho, 0, 0, c^2)
template <int NDIM, int R, typename Real, int IK>
__device__ __forceinline__ void reconstruct(const Real* __restrict__ s, int fs, int l, const Tab<Real>& T,
                                            Real gamma, int positivity, Real (&qp)[2 + NDIM],
                                            Real (&qm)[2 + NDIM]) {
    constexpr int NV = 2 + NDIM;
    constexpr int NS = 2 * R + 1;
    Real v[NV][NS];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int j = 0; j < NS; ++j) v[k][j] = s[k * fs + l + j];

    const Real rho = v[0][R], p = v[NV - 1][R];
    const Real irho = frcp(rho);
    const Real c2 = gamma * p * irho;
    const Real ic = frsq(c2);
    const Real c = c2 * ic;
    const Real ic2 = ic * ic;
    const Real a = Real(0.5) * rho * ic;
    const Real b = Real(0.5) * ic2;

    // Fields in the order that retires stencil values soonest: the shear
    // velocities, then the entropy wave (density), then the two acoustic
    // waves (normal velocity and pressure). Bitwise the same result as any
    // other order; it saves 10-24 registers (3D float64 R = 3: 139 -> 115).
    Real f[NS];
    Real acm_p, acm_m, ent_p, ent_m, acp_p, acp_m;
#pragma unroll
    for (int t = 0; t < NDIM - 1; ++t) {
#pragma unroll
        for (int j = 0; j < NS; ++j) f[j] = v[2 + t][j];
        interp<R, Real, IK>(f, T, qp[2 + t], qm[2 + t]);
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) f[j] = fma(-ic2, v[NV - 1][j], v[0][j]);
    interp<R, Real, IK>(f, T, ent_p, ent_m);
#pragma unroll
    for (int j = 0; j < NS; ++j) f[j] = fma(-a, v[1][j], b * v[NV - 1][j]);
    interp<R, Real, IK>(f, T, acm_p, acm_m);
#pragma unroll
    for (int j = 0; j < NS; ++j) f[j] = fma(a, v[1][j], b * v[NV - 1][j]);
    interp<R, Real, IK>(f, T, acp_p, acp_m);
    const Real cr = c * irho;
    qp[0] = acm_p + ent_p + acp_p;
    qm[0] = acm_m + ent_m + acp_m;
    qp[1] = cr * (acp_p - acm_p);
    qm[1] = cr * (acp_m - acm_m);
    qp[NV - 1] = c2 * (acm_p + acp_p);
    qm[NV - 1] = c2 * (acm_m + acp_m);
    if (positivity) {
        if (!(qp[0] > Real(0)) || !(qp[NV - 1] > Real(0))) {
#pragma unroll
            for (int k = 0; k < NV; ++k) qp[k] = v[k][R];
        }
        if (!(qm[0] > Real(0)) || !(qm[NV - 1] > Real(0))) {
#pragma unroll
            for (int k = 0; k < NV; ++k) qm[k] = v[k][R];
        }
    }
}

// Euler flux of a rotated primitive state, and its conserved vector.
template <int NDIM, typename Real>
__device__ __forceinline__ void flux_of(const Real (&q)[2 + NDIM], Real inv_gm1, Real (&F)[2 + NDIM],
                                        Real (&Uc)[2 + NDIM]) {
    constexpr int NV = 2 + NDIM;
    const Real r = q[0], u = q[1], p = q[NV - 1];
    Real k2 = u * u;
#pragma unroll
    for (int t = 0; t < NDIM - 1; ++t) k2 = fma(q[2 + t], q[2 + t], k2);
    const Real E = fma(p, inv_gm1, Real(0.5) * r * k2);
    const Real mu = r * u;
    F[0] = mu;
    F[1] = fma(mu, u, p);
#pragma unroll
    for (int t = 0; t < NDIM - 1; ++t) F[2 + t] = mu * q[2 + t];
    F[NV - 1] = u * (E + p);
    Uc[0] = r;
    Uc[1] = mu;
#pragma unroll
    for (int t = 0; t < NDIM - 1; ++t) Uc[2 + t] = r * q[2 + t];
    Uc[NV - 1] = E;
}

// HLLC flux (rotated frame) with Davis wave-speed estimates; at S* = 0 the left
// star state is used. Branch-free. The face takes the flux of one side K only:
// the upwind side of a supersonic face (S_L >= 0: left, S_R <= 0: right), else
// the side of the contact the face lies on. So the primitive state of K is
// selected first and only its flux and conserved vector are formed; the star
// state of K gives F = F_K + S_K (U*_K - U_K) on subsonic faces.
template <int NDIM, typename Real>
__device__ __forceinline__ void hllc(const Real (&qL)[2 + NDIM], const Real (&qR)[2 + NDIM], Real gamma,
                                     Real inv_gm1, Real (&F)[2 + NDIM]) {
    constexpr int NV = 2 + NDIM;
    const Real rL = qL[0], uL = qL[1], pL = qL[NV - 1];
    const Real rR = qR[0], uR = qR[1], pR = qR[NV - 1];
    // 1/rho_L and 1/rho_R from one reciprocal
    const Real irLR = frcp(rL * rR);
    const Real c2L = gamma * pL * (rR * irLR);
    const Real c2R = gamma * pR * (rL * irLR);
    const Real cL = c2L * frsq(c2L);
    const Real cR = c2R * frsq(c2R);
    const Real SL = fmin(uL - cL, uR - cR);
    const Real SR = fmax(uL + cL, uR + cR);
    const Real mL = rL * (SL - uL);
    const Real mR = rR * (SR - uR);
    const Real Ss = (pR - pL + uL * mL - uR * mR) * frcp(mL - mR);
    const bool sup = SL >= Real(0) || SR <= Real(0);
    const bool left = SL >= Real(0) || (SR > Real(0) && Ss >= Real(0));
    Real qK[NV], FK[NV], UK[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) qK[k] = left ? qL[k] : qR[k];
    flux_of<NDIM, Real>(qK, inv_gm1, FK, UK);
    const Real u = qK[1], p = qK[NV - 1];
    const Real S = left ? SL : SR;
    const Real m = left ? mL : mR;
    // with X = m (S - S*): m/(S - S*) = m^2/X, 1/m = (S - S*)/X and
    // 1/rho = (S - u)/m = (S - u)(S - S*)/X, all from one reciprocal
    const Real dS = S - Ss;
    const Real iX = frcp(m * dS);
    const Real fac = m * m * iX;
    const Real im = dS * iX;
    const Real ir = (S - u) * im;
    Real Us[NV];
    Us[0] = fac;
    Us[1] = fac * Ss;
#pragma unroll
    for (int t = 0; t < NDIM - 1; ++t) Us[2 + t] = fac * qK[2 + t];
    Us[NV - 1] = fac * (UK[NV - 1] * ir + (Ss - u) * (Ss + p * im));
#pragma unroll
    for (int k = 0; k < NV; ++k) F[k] = sup ? FK[k] : fma(S, Us[k] - UK[k], FK[k]);
}

template <int NDIM, int DIR, int R, typename Real, int NC>
struct SweepCfg {
    static constexpr int NV = 2 + NDIM;
    static constexpr int LEFT = run_left(NC);  // first output lane of a run
    static constexpr int TOUT = run_out(NC);   // outputs per run
    static constexpr int SLEN = WAVE + 2 * R;
    static constexpr int PITCH = SLEN | 1;
    static constexpr int WPB = sweep_wpb(NDIM, DIR, sizeof(Real) == 4);  // pencils (waves) per block
    static constexpr int THREADS = WPB * WAVE;
    static constexpr size_t IN_BYTES = sizeof(Real) * NV * WPB * PITCH;
    static constexpr int OPITCH = WPB + 1;  // padded row of the output tile (no bank conflicts)
    static constexpr size_t OUT_BYTES = (DIR == 0) ? 0 : sizeof(double) * NV * TOUT * OPITCH;
    static constexpr size_t SMEM = IN_BYTES > OUT_BYTES ? IN_BYTES : OUT_BYTES;
};

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}

// DPP move of a double (both halves with the same control): lanes the row mask
// leaves out keep `old`; with bound_ctrl a lane whose source is out of range
// reads 0.
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ double dpp_f64(double x, double old) {
    const long long b = __double_as_longlong(x), o = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xF, BOUND);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, ROW_MASK, 0xF, BOUND);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Max over the wave of non-negative doubles, returned to every lane. Row shifts
// by 1, 2, 4, 8 (out-of-row sources read 0, the identity here) leave each row's
// max in its lane 15; row_bcast:15 and row_bcast:31 carry those across rows into
// lane 63. Registers only, no LDS round trips.
__device__ __forceinline__ double wave_max_nonneg(double v) {
    v = fmax(v, dpp_f64<0x111, 0xF, true>(v, v));  // row_shr:1
    v = fmax(v, dpp_f64<0x112, 0xF, true>(v, v));  // row_shr:2
    v = fmax(v, dpp_f64<0x114, 0xF, true>(v, v));  // row_shr:4
    v = fmax(v, dpp_f64<0x118, 0xF, true>(v, v));  // row_shr:8
    v = fmax(v, dpp_f64<0x142, 0xA, false>(v, v)); // row_bcast:15 into rows 1, 3
    v = fmax(v, dpp_f64<0x143, 0xC, false>(v, v)); // row_bcast:31 into rows 2, 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Physical check and CFL speed sum_d (|u_d| + c)/dx_d of one cell's conserved
// values o (ix: 1/dx per axis). ok: rho > 0 and p > 0 (false for NaN). The sound
// speed comes from the reciprocal square root (to an ulp or two); a cell whose
// speed is NaN reads as infinitely fast. The finishing sweep of stage 3 and the
// CFL-speed kernel both call this, so they give a state the same speed.
template <int NDIM>
__device__ __forceinline__ double cell_speed(const double (&o)[2 + NDIM], double gamma, const double* ix, bool& ok,
                                             bool want_speed) {
    constexpr int NV = 2 + NDIM;
    const double rho = o[0];
    const double irho = frcp(rho);
    double ke = 0.0, vel[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int dd = 0; dd < NDIM; ++dd) {
        vel[dd] = o[1 + dd] * irho;
        ke += vel[dd] * o[1 + dd];
    }
    const double p = (gamma - 1.0) * (o[NV - 1] - 0.5 * ke);
    ok = rho > 0.0 && p > 0.0;
    if (!want_speed) return 0.0;
    const double c2 = gamma * p * irho;
    const double c = c2 * frsq(c2);
    double s = 0.0;
#pragma unroll
    for (int dd = 0; dd < NDIM; ++dd) s += (fabs(vel[dd]) + c) * ix[dd];
    return (s != s) ? (double)INFINITY : s;
}

// Finish one cell. FIN = false: accumulate the direction's contribution into
// dU. FIN = true (last direction of an RK stage): form the stage output
// (SSP-RK3, Shu-Osher form), check it is physical and, in stage 3, track the
// CFL speed of the new state.
template <int NDIM, bool FIN, typename Real>
__device__ __forceinline__ void finish_cell(const SweepArgs<Real>& a, long long cell, const double (&d)[2 + NDIM],
                                            const double (&pd)[2 + NDIM], const double (&pu)[2 + NDIM],
                                            const double (&pn)[2 + NDIM], double dt, double& spd) {
    constexpr int NV = 2 + NDIM;
    const long long nc = a.ncell;
    if (!FIN) {
#pragma unroll
        for (int k = 0; k < NV; ++k) a.dU[k * nc + cell] = a.first ? d[k] : pd[k] + d[k];
        return;
    }
    double o[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double L = a.first ? d[k] : pd[k] + d[k];
        o[k] = fma(dt, L, pu[k]);  // the stage input advanced by dt L
    }
    // Shu-Osher weights of stages 2 and 3 (3/4 U^n + 1/4 adv, 1/3 U^n + 2/3 adv),
    // one uniform branch for all components
    if (a.stage != 1) {
        const double cn = a.stage == 2 ? 0.75 : 1.0 / 3.0, cu = a.stage == 2 ? 0.25 : 2.0 / 3.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) o[k] = fma(cn, pn[k], cu * o[k]);
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) a.Uout[k * nc + cell] = o[k];
    bool ok;
    const double s = cell_speed<NDIM>(o, a.gamma, a.inv_dx_all, ok, a.stage == 3);
    if (!ok) {
        atomicOr(&a.ctl->err, 1);
        atomicMin(&a.ctl->bad_cell, cell);
    }
    if (a.stage == 3) spd = s;
}

// XCD-aware block order. Workgroups are dealt to the 8 XCDs round-robin by
// index; renumber them so that each XCD gets one contiguous range of logical
// blocks. Logical order is "band-major" in every direction (rows for x sweeps,
// runs along y / z for y / z sweeps), so an XCD keeps working on roughly the
// same slab of the grid in every sweep, and the slab's stage states and
// accumulator stay in that XCD's L2 between kernels.
__device__ __forceinline__ long long xcd_logical_block() {
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned q8 = nb >> 3, r8 = nb & 7u, xcd = b & 7u;
    return (long long)(xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3));
}

// The first sweep of a step (block 0): mark the step as running (or not), store
// its dt for the sweeps that finish a stage, and clear the next speed slot.
template <bool FIN>
__device__ __forceinline__ void mark_step(Ctl* c, bool go, long long nstep, double t0, double dt) {
    c->started = go ? nstep : -1;
    if (go) {
        c->dt_step[nstep & 1] = FIN ? dt : step_dt(c, nstep, t0);
#pragma unroll
        for (int x = 0; x < 8; ++x) c->xcd[x].speed[(nstep + 1) & 1] = 0ull;
    }
}

// One block of a sweep: logical block L of the problem's blocks.
template <int NDIM, int DIR, int R, typename Real, bool FIN, int IK, bool BCG, int NC>
__device__ __forceinline__ void sweep_block(const SweepArgs<Real>& a, const long long L, unsigned char* smem,
                                            unsigned long long* sred) {
    using C = SweepCfg<NDIM, DIR, R, Real, NC>;
    constexpr int NV = C::NV, WPB = C::WPB, PITCH = C::PITCH, SLEN = C::SLEN, THREADS = C::THREADS;
    constexpr int LEFT = C::LEFT, TOUT = C::TOUT;
    // float64 sweeps request their epilogue operands (and, in x sweeps, their
    // own cell's conserved values) after the reconstruction rather than before
    // it: held through it, those registers cost the float64 finishing sweep an
    // occupancy level (111 against 87 VGPRs for 2D R = 2) and the 2D R = 3 y
    // sweep another (103 against 95), which outweighs the shorter time the
    // loads have to arrive (the 3D y sweep gains 7 % at equal occupancy).
    // float32 sweeps gain nothing either way and keep the early requests.
    constexpr bool LATE = sizeof(Real) == 8;
    Real* sV = reinterpret_cast<Real*>(smem);
    double* sO = reinterpret_cast<double*>(smem);

    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int w = tid / WAVE;
    const int N = a.n[DIR];
    // Block geometry in 32-bit arithmetic: logical blocks number below 2^31
    // (checked at launch). Segment seg of a pencil covers cells s0 .. s0 + tseg
    // - 1; the first N % nseg segments take one cell more than the others.
    const unsigned Lu = (unsigned)L, nseg = (unsigned)a.nseg;
    unsigned seg, grp, other = 0;  // grp: row group (DIR 0) or x group; other: z (DIR 1) or y (DIR 2)
    const unsigned nxb = ((unsigned)a.n[0] + WPB - 1) / WPB;
    if (DIR == 0) {
        seg = Lu % nseg;
        grp = Lu / nseg;
    } else if (DIR == 1) {
        grp = Lu % nxb;
        const unsigned t = Lu / nxb;
        seg = t % nseg;
        other = t / nseg;
    } else {
        grp = Lu % nxb;
        const unsigned t = Lu / nxb;
        other = t % (unsigned)a.n[1];
        seg = t / (unsigned)a.n[1];
    }
    const unsigned sq = (unsigned)N / nseg, sr = (unsigned)N % nseg;
    const int s0 = (int)(seg * sq + (seg < sr ? seg : sr));
    const int tseg = (int)(sq + (seg < sr ? 1u : 0u));
    const int sbase = s0 - LEFT - R;
    const long long nc = a.ncell;
    const double gamma = a.gamma;

    // ---- pencil geometry ----------------------------------------------------
    long long stride;
    long long blk_base;   // cell of column 0 at s = 0
    int ncol_valid;       // pencils of this block that exist
    if (DIR == 0) {
        stride = 1;
        const long long nrows = (long long)a.n[1] * a.n[2];
        const long long row0 = (long long)grp * WPB;
        blk_base = row0 * a.n[0];
        ncol_valid = (int)((nrows - row0) < WPB ? (nrows - row0) : WPB);
    } else {
        const int xb = (int)grp * WPB;
        stride = (DIR == 1) ? (long long)a.n[0] : (long long)a.n[0] * a.n[1];
        blk_base = xb + (long long)other * (DIR == 1 ? (long long)a.n[0] * a.n[1] : (long long)a.n[0]);
        ncol_valid = (a.n[0] - xb) < WPB ? (a.n[0] - xb) : WPB;
    }
    // column c of the block starts at blk_base + c * cstride
    const long long cstride = (DIR == 0) ? (long long)a.n[0] : 1;

    // ---- the stencil tile's float64 conserved values ---------------------------
    // Every tile load of a thread is issued before any of them is used, so a
    // block waits for one round trip before it computes.
    // x sweeps: pass 0, lane l of wave w loads tile position l + R of row w (its
    // own cell); pass 1, the first WPB * 2R threads (all in wave 0) load the 2R
    // halo positions of every row (0 .. R-1 and 64 + R .. 64 + 2R - 1), so the
    // other waves skip the pass.
    // y/z sweeps: tile rows are dealt rotated by LEFT + R, so that in pass 0
    // thread t loads the cell it finishes in the epilogue (row t / WPB of the
    // output tile); pass 1 covers the remaining 2R rows.
    constexpr int FS = WPB * PITCH;
    static_assert(WPB * 2 * R <= WAVE, "the halo pass fits one wave");
    int tcol[2], tpos[2];
    bool tact1;
    if (DIR == 0) {
        tcol[0] = w;
        tpos[0] = lane + R;
        const int j = tid % (2 * R);
        tcol[1] = tid / (2 * R);
        tpos[1] = j < R ? j : WAVE + j;
        tact1 = tid < WPB * 2 * R;
    } else {
        constexpr int ROWS = THREADS / WPB;
        static_assert(SLEN <= 2 * ROWS, "two passes cover the tile");
        tcol[0] = tcol[1] = tid % WPB;
        const int p = tid / WPB;
        tpos[0] = (p + LEFT + R) % SLEN;
        tpos[1] = (p + ROWS + LEFT + R) % SLEN;
        tact1 = p + ROWS < SLEN;
    }
    const bool tcol_ok[2] = {tcol[0] < ncol_valid, tcol[1] < ncol_valid};
    double u[2][NV];
    bool flip[2] = {false, false};
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (tcol_ok[r] && (r == 0 || tact1)) {
            const int src = BCG ? ghost_src(sbase + tpos[r], N, a.bc[0], a.bc[1], flip[r]) : wrap(sbase + tpos[r], N);
            const long long cell = blk_base + tcol[r] * cstride + (long long)src * stride;
#pragma unroll
            for (int k = 0; k < NV; ++k) u[r][k] = a.U[k * nc + cell];
        }
    }

    // ---- step control: read after the tile loads are in flight, so the two
    // round trips overlap (a halted step's loads are simply dropped)
    double t0 = 0.0, dt = 0.0;
    long long nstep = 0;
    if (a.stage > 0) {
        const bool go = step_go<FIN>(a.ctl, FIN && a.stage == 3, FIN && a.step_start, t0, dt, nstep);
        if (a.step_start && L == 0 && threadIdx.x == 0) mark_step<FIN>(a.ctl, go, nstep, t0, dt);
        if (!go) return;
    }

    // ---- the cell each thread finishes ---------------------------------------
    // Each thread finishes at most one cell: its own lane's cell in x sweeps,
    // one cell of the transposed output tile in y / z sweeps.
    static_assert(DIR == 0 || TOUT * WPB <= THREADS, "one epilogue cell per thread");
    long long ecell = -1;
    if (DIR == 0) {
        if (w < ncol_valid && lane >= LEFT && lane < LEFT + tseg)
            ecell = blk_base + w * cstride + (s0 + lane - LEFT);
    } else {
        const int row = tid / WPB, c = tid % WPB;
        if (row < tseg && c < ncol_valid) ecell = blk_base + c * cstride + (long long)(s0 + row) * stride;
    }
    double pd[NV], pu[NV], pn[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) pd[k] = pu[k] = pn[k] = 0.0;

    // ---- convert to rotated primitive variables and stage in LDS --------------
    // Pass 0 of the thread that finishes a cell loaded that very cell; its
    // float64 conserved values are kept for the epilogue.
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (r == 1 && !tact1) break;
        double q[NV];
        if (tcol_ok[r]) {
            if (FIN && !LATE && r == 0 && ecell >= 0) {
#pragma unroll
                for (int k = 0; k < NV; ++k) pu[k] = u[0][k];
            }
            if (BCG && flip[r]) u[r][1 + DIR] = -u[r][1 + DIR];
            cons_to_rot<NDIM, DIR>(u[r], gamma, q);
        } else {
#pragma unroll
            for (int k = 0; k < NV; ++k) q[k] = (k == 0 || k == NV - 1) ? 1.0 : 0.0;
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) sV[k * FS + tcol[r] * PITCH + tpos[r]] = (Real)q[k];
    }

    // ---- epilogue operands: requested now, they arrive while the sweep computes
    // (each uniform condition tested once, outside the loops over components)
    if (!LATE && ecell >= 0) {
        if (!a.first) {
#pragma unroll
            for (int k = 0; k < NV; ++k) pd[k] = a.dU[k * nc + ecell];
        }
        if (FIN && a.stage >= 2) {
#pragma unroll
            for (int k = 0; k < NV; ++k) pn[k] = a.Un[k * nc + ecell];
        }
    }

    __syncthreads();

    // ---- per-lane reconstruction, face flux, correction, difference ----------
    double dcons[NV];
    {
        const Real g = (Real)gamma;
        const Real inv_gm1 = (Real)a.inv_gm1;
        Real qp[NV], qm[NV];
        reconstruct<NDIM, R, Real, IK>(sV + w * PITCH, FS, lane, a.tab, g, a.positivity, qp, qm);
        if (LATE && ecell >= 0) {
            if (!a.first) {
#pragma unroll
                for (int k = 0; k < NV; ++k) pd[k] = a.dU[k * nc + ecell];
            }
            if (FIN && a.stage >= 2) {
#pragma unroll
                for (int k = 0; k < NV; ++k) pn[k] = a.Un[k * nc + ecell];
            }
            if (FIN) {
#pragma unroll
                for (int k = 0; k < NV; ++k) pu[k] = a.U[k * nc + ecell];
            }
        }
        Real qR[NV], F[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) qR[k] = lane_next(qm[k]);
        hllc<NDIM, Real>(qp, qR, g, inv_gm1, F);
        // f^ = F + alpha (F_{-1} - 2F + F_{+1}) + beta (F_{-2} - 4F_{-1} + 6F - 4F_{+1} + F_{+2})
        //       [+ g (F_{-3} - 6F_{-2} + 15F_{-1} - 20F + 15F_{+1} - 6F_{+2} + F_{+3})],
        // alpha = -1/24, beta = 3/640, g = -5/7168 (NC = 3 only), gathered by
        // neighbour distance
        constexpr double AL = -1.0 / 24.0, BE = 3.0 / 640.0, G6 = NC == 3 ? -5.0 / 7168.0 : 0.0;
        const Real c0 = Real(1.0 - 2.0 * AL + 6.0 * BE - 20.0 * G6);
        const Real c1 = Real(AL - 4.0 * BE + 15.0 * G6);
        const Real c2 = Real(BE - 6.0 * G6);
        const Real c3 = Real(G6);
        // This lane's face is x_{i+1/2} of cell i. At a reflecting wall the mirror
        // ghosts make the fluxes of mass, tangential momentum and energy vanish
        // (and the correction terms with them, by antisymmetry) up to rounding;
        // they are set to exactly zero so that float32 sweeps conserve mass and
        // energy in a closed box to float64 rounding as well.
        const int icell = s0 - LEFT + lane;
        const bool wall = BCG && ((a.bc[0] == 2 && icell == -1) || (a.bc[1] == 2 && icell == N - 1));
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const Real fm1 = lane_prev(F[k]), fm2 = lane_prev(fm1);
            const Real fp1 = lane_next(F[k]), fp2 = lane_next(fp1);
            Real far = c2 * (fm2 + fp2);
            if constexpr (NC == 3) far = fma(c3, lane_prev(fm2) + lane_next(fp2), far);
            const Real fh = (wall && k != 1) ? Real(0) : fma(c0, F[k], fma(c1, fm1 + fp1, far));
            const Real fhm = lane_prev(fh);
            dcons[cons_slot<NDIM, DIR>(k)] = -((double)fh - (double)fhm) * a.inv_dx;
        }
    }

    double spd = 0.0;  // this lane's CFL speed (stage 3 of a finishing sweep)
    const bool lane_out = lane >= LEFT && lane < LEFT + tseg;
    if (DIR == 0) {
        if (ecell >= 0) finish_cell<NDIM, FIN, Real>(a, ecell, dcons, pd, pu, pn, dt, spd);
    } else {
        __syncthreads();  // every wave is done reading the stencil tile
        if (lane_out) {
#pragma unroll
            for (int k = 0; k < NV; ++k) sO[(k * TOUT + (lane - LEFT)) * C::OPITCH + w] = dcons[k];
        }
        __syncthreads();
        if (ecell >= 0) {
            const int row = tid / WPB, c = tid % WPB;
            double d[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) d[k] = sO[(k * TOUT + row) * C::OPITCH + c];
            finish_cell<NDIM, FIN, Real>(a, ecell, d, pd, pu, pn, dt, spd);
        }
    }
    if (FIN && a.stage == 3) {
        // CFL speed of the new state into the next step's slot (one atomic per
        // block, no return value), and block 0 closes the step by writing the
        // next step state into the older record (see Ctl).
        // non-negative doubles order like their bit images
        const double wmax = wave_max_nonneg(spd);
        if (lane == 0) sred[w] = (unsigned long long)__double_as_longlong(wmax);
        __syncthreads();
        if (tid == 0) {
            unsigned long long m = sred[0];
#pragma unroll
            for (int i = 1; i < WPB; ++i) m = sred[i] > m ? sred[i] : m;
            Ctl* c = a.ctl;
            atomicMax(&c->xcd[blockIdx.x & 7u].speed[(nstep + 1) & 1], m);
            if (L == 0) {
                const int older = (c->rec[0].nsteps == nstep) ? 1 : 0;
                c->rec[older].t = t0 + dt;
                c->rec[older].dt = dt;
                c->rec[older].nsteps = nstep + 1;
            }
        }
    }
}

template <int NDIM, int DIR, int R, typename Real, bool FIN, int IK, bool BCG, int NC>
__global__ void __launch_bounds__((SweepCfg<NDIM, DIR, R, Real, NC>::THREADS))
sweep_kernel(const SweepArgs<Real> a) {
    using C = SweepCfg<NDIM, DIR, R, Real, NC>;
    __shared__ __attribute__((aligned(16))) unsigned char smem[C::SMEM];
    __shared__ unsigned long long sred[C::WPB];
    sweep_block<NDIM, DIR, R, Real, FIN, IK, BCG, NC>(a, xcd_logical_block(), smem, sred);
}

// Batched sweep over many independent problems (same ndim, R, precision and
// tables). Logical blocks are laid out problem after problem; the launch's
// work table (BatchDir, in device memory) holds the problems' descriptors,
// the owner of every logical block and their count, one hardware block per
// logical block. The host changes the set by rewriting the table with
// stream-ordered copies and the grid of the captured launch in place, so a
// captured graph of batched steps serves every set of the same kinds of
// problems. Every block runs exactly the code of the single-problem sweep on
// its own problem's data, so a problem's result does not depend on what else
// is in the batch.
template <int NDIM, int DIR, int R, typename Real, bool FIN, int IK, bool BCG, int NC>
__global__ void __launch_bounds__((SweepCfg<NDIM, DIR, R, Real, NC>::THREADS))
sweep_batch_kernel(const BatchArgs<Real> ba) {
    using C = SweepCfg<NDIM, DIR, R, Real, NC>;
    __shared__ __attribute__((aligned(16))) unsigned char smem[C::SMEM];
    __shared__ unsigned long long sred[C::WPB];
    const BatchDir* D = ba.dir;
    const long long Lg = xcd_logical_block();
    if (Lg >= D->nblocks) return;   // a grid of one block for an empty group
    const ProbDesc& P = D->probs[D->owner[Lg]];
    SweepArgs<Real> a;
    a.U = P.U;
    a.Un = P.Un;
    a.dU = P.dU;
    a.Uout = P.Uout;
    a.ctl = P.ctl;
    a.n[0] = P.n[0];
    a.n[1] = P.n[1];
    a.n[2] = P.n[2];
    a.nseg = P.nseg;
    a.ncell = P.ncell;
    a.inv_dx = P.inv_dx;
    a.inv_dx_all[0] = P.inv_dx_all[0];
    a.inv_dx_all[1] = P.inv_dx_all[1];
    a.inv_dx_all[2] = P.inv_dx_all[2];
    a.gamma = P.gamma;
    a.inv_gm1 = P.inv_gm1;
    a.positivity = P.positivity;
    a.bc[0] = P.bc[0];
    a.bc[1] = P.bc[1];
    a.first = ba.first;
    a.stage = ba.stage;
    a.step_start = ba.step_start;
    a.tab = ba.tab;
    sweep_block<NDIM, DIR, R, Real, FIN, IK, BCG, NC>(a, Lg - P.block0, smem, sred);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// A launch of kernel K: the single-problem sweep (grid from the problem's
// geometry) or the batched sweep (grid given by the caller).
template <int NDIM, int DIR, int R, typename Real, bool FIN, int IK, bool BCG, int NC>
hipError_t launch_one(const void* args, long long blocks, bool batch, hipStream_t s) {
    using C = SweepCfg<NDIM, DIR, R, Real, NC>;
    if (batch) {
        const BatchArgs<Real>& a = *static_cast<const BatchArgs<Real>*>(args);
        if (blocks <= 0 || blocks > INT_MAX) return hipErrorInvalidValue;
        hipLaunchKernelGGL((sweep_batch_kernel<NDIM, DIR, R, Real, FIN, IK, BCG, NC>), dim3((unsigned)blocks),
                           dim3(C::THREADS), 0, s, a);
        return hipGetLastError();
    }
    const SweepArgs<Real>& a = *static_cast<const SweepArgs<Real>*>(args);
    long long groups;
    if (DIR == 0) {
        groups = ((long long)a.n[1] * a.n[2] + C::WPB - 1) / C::WPB;
    } else {
        const long long nxb = (a.n[0] + C::WPB - 1) / C::WPB;
        groups = nxb * (DIR == 1 ? a.n[2] : a.n[1]);
    }
    blocks = groups * a.nseg;
    if (blocks <= 0 || blocks > INT_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sweep_kernel<NDIM, DIR, R, Real, FIN, IK, BCG, NC>), dim3((unsigned)blocks), dim3(C::THREADS),
                       0, s, a);
    return hipGetLastError();
}

// A finishing kernel exists only for x, the last direction of a stage.
template <int NDIM, int R, typename Real, int IK, bool BCG, int NC>
hipError_t launch_dir(const LaunchSel& k, const void* args, long long blocks, hipStream_t s) {
    if (k.fin) {
        if (k.dir != 0) return hipErrorInvalidValue;
        return launch_one<NDIM, 0, R, Real, true, IK, BCG, NC>(args, blocks, k.batch, s);
    }
    if (k.dir == 0) return launch_one<NDIM, 0, R, Real, false, IK, BCG, NC>(args, blocks, k.batch, s);
    if (NDIM >= 2 && k.dir == 1)
        return launch_one<NDIM, (NDIM >= 2 ? 1 : 0), R, Real, false, IK, BCG, NC>(args, blocks, k.batch, s);
    if (NDIM == 3 && k.dir == 2)
        return launch_one<NDIM, (NDIM == 3 ? 2 : 0), R, Real, false, IK, BCG, NC>(args, blocks, k.batch, s);
    return hipErrorInvalidValue;
}

template <int NDIM, int R, typename Real, int IK, int NC>
hipError_t launch_bcg(const LaunchSel& k, const void* args, long long blocks, hipStream_t s) {
    return k.bcg ? launch_dir<NDIM, R, Real, IK, true, NC>(k, args, blocks, s)
                 : launch_dir<NDIM, R, Real, IK, false, NC>(k, args, blocks, s);
}

// Indicator kinds: 0 for R = 1..3, 1 (Jiang-Shu) for R = 1, 2, 2 for R = 1..3,
// 3 (adaptive order) for R = 2, 3. The three-term flux correction exists for
// indicator kind 0 only.
template <int NDIM, typename Real, int IK, int NC>
hipError_t launch_rk(const LaunchSel& k, const void* args, long long blocks, hipStream_t s) {
    switch (k.R) {
        case 1:
            if constexpr (IK != 3) return launch_bcg<NDIM, 1, Real, IK, NC>(k, args, blocks, s);
            return hipErrorInvalidValue;
        case 2: return launch_bcg<NDIM, 2, Real, IK, NC>(k, args, blocks, s);
        case 3:
            if constexpr (IK != 1) return launch_bcg<NDIM, 3, Real, IK, NC>(k, args, blocks, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <int NDIM, typename Real>
hipError_t launch_r(const LaunchSel& k, const void* args, long long blocks, hipStream_t s) {
    if (k.nc == 3) {
        if (k.ik != 0) return hipErrorInvalidValue;
        return launch_rk<NDIM, Real, 0, 3>(k, args, blocks, s);
    }
    if (k.nc != 2) return hipErrorInvalidValue;
    switch (k.ik) {
        case 0: return launch_rk<NDIM, Real, 0, 2>(k, args, blocks, s);
        case 1: return launch_rk<NDIM, Real, 1, 2>(k, args, blocks, s);
        case 2: return launch_rk<NDIM, Real, 2, 2>(k, args, blocks, s);
        case 3: return launch_rk<NDIM, Real, 3, 2>(k, args, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gpw
