"""GP-WENO pre-simulation tables, computed in arbitrary precision (mpmath).

TEST INFRASTRUCTURE ONLY: part of the CPU oracle. Only ``tests/``, the smoke
check and the benchmark's CPU-baseline leg may use it; the product path never does.

Follows Sec. 4 "A Stepwise Description of GP-WENO", step 1 (pre-simulation):
  (b) covariance matrices K (Eq. (kmat)) on the 2R+1 stencil S_R and K_m on each
      sub-stencil S_m, prediction vectors k_* (Eq. (kstar)), GP weights
      w_*^T = k_*^T K^{-1} and w_m^T = k_{*,m}^T K_m^{-1} (Sec. 3.2, Eq. (q-intrp));
  (c) optimal linear weights gamma as the least-squares solution of the
      (2R+1)x(R+1) system M gamma = w_* (Sec. 3.3, Eqs. (gamm-system), (M-mat));
  (d) the eigensystem of K_m built with the second length scale sigma
      (Sec. 3.4), stored as P_i = v_i / sqrt(lambda_i) (Eq. (beta-eigen)).

Coordinates are in units of the grid spacing: stencil nodes at the integers
-R..R relative to the centre cell, the prediction point at x_* = +1/2 or -1/2.
The squared-exponential kernel (Eq. (se)) is used with Sigma = 1 (it cancels).

Reading (the paper gives no precision for this step and only warns about a
"singularity issue" for large ell/dx): K is very badly conditioned at the
usual ell = 12 dx (condition number ~1e5, 6e9, 8e13 for R = 1, 2, 3), so the
tables are computed with 60 significant digits and rounded to float64 at the end.
No normalisation of w or gamma is applied: gamma is the plain least-squares
solution, as stated in Sec. 3.3.

Sub-stencil indexing: m = 0..R (the paper's m = 1..R+1); sub-stencil m holds
the nodes m-R .. m, i.e. entries m .. m+R of the 2R+1 stencil vector.
"""
from __future__ import annotations

import functools
from fractions import Fraction

import mpmath as mp
import numpy as np

DEFAULT_DPS = 60


def _se(a, b, ell):
    """Squared-exponential kernel with Sigma = 1 (Eq. (se), Eq. (kmat))."""
    return mp.exp(-((a - b) ** 2) / (2 * ell * ell))


def _kernel_matrix(nodes, ell):
    n = len(nodes)
    K = mp.matrix(n, n)
    for j in range(n):
        for k in range(n):
            K[j, k] = _se(nodes[j], nodes[k], ell)
    return K


def _kstar(nodes, xstar, ell):
    return mp.matrix([_se(xstar, x, ell) for x in nodes])


@functools.lru_cache(maxsize=256)
def gp_tables_mp(R: int, ell: str, sigma: str, dps: int = DEFAULT_DPS):
    """All tables as mpmath numbers. ``ell`` and ``sigma`` are decimal strings in
    units of dx (strings so that the cache key is exact).

    Returns a dict with keys
      'wstar+', 'wstar-' : lists (2R+1) of full-stencil weights at x_* = +-1/2
      'w+', 'w-'         : lists [m][j], m, j = 0..R, sub-stencil weights
      'gamma+', 'gamma-' : lists (R+1) of linear weights
      'P'                : list [i][j] of rows P_i = v_i / sqrt(lambda_i) of K_m(sigma)
      'lambda'           : eigenvalues of K_m(sigma)
      'cond'             : condition number estimate of K(ell)
    """
    with mp.workdps(dps):
        ellm = mp.mpf(ell)
        sigm = mp.mpf(sigma)
        nodes = [mp.mpf(j) for j in range(-R, R + 1)]
        out = {}
        K = _kernel_matrix(nodes, ellm)
        out["cond"] = mp.cond(K)
        for sign, key in ((+1, "+"), (-1, "-")):
            xstar = mp.mpf(sign) / 2
            # step 1(b): global-stencil and sub-stencil GP weights
            wstar = mp.lu_solve(K, _kstar(nodes, xstar, ellm))
            wsub = []
            for m in range(R + 1):
                sub = nodes[m : m + R + 1]
                Km = _kernel_matrix(sub, ellm)
                wsub.append(list(mp.lu_solve(Km, _kstar(sub, xstar, ellm))))
            # step 1(c): M gamma = w_*, column n carries w_n in rows n .. n+R
            M = mp.zeros(2 * R + 1, R + 1)
            for n in range(R + 1):
                for j in range(R + 1):
                    M[n + j, n] = wsub[n][j]
            gam, _res = mp.qr_solve(M, wstar)
            out["wstar" + key] = list(wstar)
            out["w" + key] = wsub
            out["gamma" + key] = list(gam)
        # step 1(d): one eigensystem of K_m(sigma), identical for every m on a uniform grid
        P, lam = gp_beta_rows_mp(R, sigma, dps)
        out["P"] = P
        out["lambda"] = lam
        return out


@functools.lru_cache(maxsize=64)
def gp_beta_rows_mp(R: int, sigma: str, dps: int = DEFAULT_DPS):
    """Rows P_i = v_i / sqrt(lambda_i) of the eigensystem of K_m(sigma) (Sec. 3.4,
    Eq. (beta-eigen)), so that beta_m = sum_i (P_i . f_m)^2. ``sigma`` is a decimal
    string in units of dx. Returns (P as list [i][j], eigenvalues)."""
    with mp.workdps(dps):
        nodes = [mp.mpf(j) for j in range(R + 1)]
        Ks = _kernel_matrix(nodes, mp.mpf(sigma))
        lam, Q = mp.eigsy(Ks)
        P = [[Q[j, i] / mp.sqrt(lam[i]) for j in range(R + 1)] for i in range(R + 1)]
        return P, list(lam)


def _dec(x) -> str:
    """Exact decimal string for a float (repr round-trips)."""
    return repr(float(x))


def gp_tables(R: int, ell_over_dx: float, sigma_over_dx: float, dps: int = DEFAULT_DPS):
    """Float64 tables for the C oracle. Arrays are padded to 4x4 / 4 entries."""
    t = gp_tables_mp(R, _dec(ell_over_dx), _dec(sigma_over_dx), dps)
    wp = np.zeros((4, 4))
    wm = np.zeros((4, 4))
    gp = np.zeros(4)
    gm = np.zeros(4)
    P = np.zeros((4, 4))
    for m in range(R + 1):
        gp[m] = float(t["gamma+"][m])
        gm[m] = float(t["gamma-"][m])
        for j in range(R + 1):
            wp[m, j] = float(t["w+"][m][j])
            wm[m, j] = float(t["w-"][m][j])
            P[m, j] = float(t["P"][m][j])
    return {"w+": wp, "w-": wm, "gamma+": gp, "gamma-": gm, "P": P,
            "wstar+": np.array([float(v) for v in t["wstar+"]]),
            "wstar-": np.array([float(v) for v in t["wstar-"]])}


# ----------------------------------------------------------------------------
# Polynomial WENO interpolation (the paper's comparison schemes, Sec. 6.2,
# Table (weno-vortex)): exact rational arithmetic.
# ----------------------------------------------------------------------------
def _pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _pder(a):
    return [k * a[k] for k in range(1, len(a))] or [Fraction(0)]


def _peval(a, x):
    return sum(c * x ** k for k, c in enumerate(a))


def _pint(a, lo, hi):
    return sum(c * (hi ** (k + 1) - lo ** (k + 1)) / (k + 1) for k, c in enumerate(a))


def _lagrange_basis(nodes):
    """Coefficients (ascending powers) of the Lagrange basis polynomials."""
    basis = []
    for j, xj in enumerate(nodes):
        p = [Fraction(1)]
        for k, xk in enumerate(nodes):
            if k != j:
                p = _pmul(p, [Fraction(-xk, xj - xk), Fraction(1, xj - xk)])
        basis.append(p)
    return basis


def _solve_exact(A, b):
    """Gauss-Jordan elimination on Fractions (A square, non-singular)."""
    n = len(A)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


@functools.lru_cache(maxsize=8)
def poly_weno_tables_exact(R: int):
    """Tables of polynomial WENO interpolation of point values (FD-Prim), exact.

    Nodes at the integers -R..R, sub-stencil m holding nodes m-R..m, prediction
    points x_* = +1/2 and -1/2 (as for the GP tables).
      'w+', 'w-'         : [m][j] Lagrange interpolation weights on S_m at x_*;
      'wstar+', 'wstar-' : the same on the whole stencil;
      'gamma+', 'gamma-' : linear weights, the exact solution of M gamma = w_*
                           (the same system as Eq. (gamm-system), which is
                           consistent for polynomial weights);
      'B'                : [m][i][j] smoothness-indicator quadratic forms of the
                           Jiang-Shu type, beta_m = f_m^T B_m f_m: the sum over
                           derivative orders l = 1..R of the integral over the
                           centre cell [-1/2, 1/2] of the squared l-th derivative
                           of the interpolating polynomial on S_m (grid spacing 1,
                           so the dx^(2l-1) scale factors are 1).
    """
    nodes = list(range(-R, R + 1))
    out = {}
    for sign, key in ((1, "+"), (-1, "-")):
        xs = Fraction(sign, 2)
        wstar = [_peval(p, xs) for p in _lagrange_basis(nodes)]
        wsub = [[_peval(p, xs) for p in _lagrange_basis(nodes[m : m + R + 1])] for m in range(R + 1)]
        M = [[Fraction(0)] * (R + 1) for _ in range(2 * R + 1)]
        for n in range(R + 1):
            for j in range(R + 1):
                M[n + j][n] = wsub[n][j]
        MtM = [[sum(M[r][a] * M[r][b] for r in range(2 * R + 1)) for b in range(R + 1)] for a in range(R + 1)]
        Mtw = [sum(M[r][a] * wstar[r] for r in range(2 * R + 1)) for a in range(R + 1)]
        gam = _solve_exact(MtM, Mtw)
        for r in range(2 * R + 1):
            if sum(M[r][a] * gam[a] for a in range(R + 1)) != wstar[r]:
                raise ArithmeticError("polynomial linear-weight system is not consistent")
        out["wstar" + key] = wstar
        out["w" + key] = wsub
        out["gamma" + key] = gam
    B = []
    half = Fraction(1, 2)
    for m in range(R + 1):
        basis = _lagrange_basis(nodes[m : m + R + 1])
        Bm = [[Fraction(0)] * (R + 1) for _ in range(R + 1)]
        ders = [basis]
        for _ in range(R):
            ders.append([_pder(p) for p in ders[-1]])
        for l in range(1, R + 1):
            for i in range(R + 1):
                for j in range(R + 1):
                    Bm[i][j] += _pint(_pmul(ders[l][i], ders[l][j]), -half, half)
        B.append(Bm)
    out["B"] = B
    return out


SCHEMES = ("gp-weno", "weno-js", "weno-gp")


def scheme_tables(scheme: str, R: int, ell_over_dx: float, sigma_over_dx: float, dps: int = DEFAULT_DPS):
    """Float64 tables for the C oracle, for one of three interpolation schemes:

      'gp-weno' : GP weights and linear weights, GP smoothness indicators
                  (the paper's method);
      'weno-js' : polynomial weights and linear weights, Jiang-Shu smoothness
                  indicators (the classical comparison scheme, R = 1, 2);
      'weno-gp' : polynomial weights and linear weights, GP smoothness
                  indicators (the hybrid of Sec. 6.2, Table (weno-vortex)).

    All three use the nonlinear weights of Eq. (weights) with p = 2, eps = 1e-36.
    'beta_form' is 'P' (beta = sum_i (P_i . f)^2) or 'B' (beta = f^T B_m f).
    """
    if scheme not in SCHEMES:
        raise ValueError(scheme)
    if scheme == "gp-weno":
        t = gp_tables(R, ell_over_dx, sigma_over_dx, dps)
        t["beta_form"] = "P"
        t["B"] = np.zeros((4, 4, 4))
        return t
    if scheme == "weno-js" and R not in (1, 2):
        raise ValueError("WENO-JS smoothness indicators are defined here for R = 1, 2")
    e = poly_weno_tables_exact(R)
    t = {k: np.zeros((4, 4)) for k in ("w+", "w-", "P")}
    t["gamma+"] = np.zeros(4)
    t["gamma-"] = np.zeros(4)
    t["B"] = np.zeros((4, 4, 4))
    for m in range(R + 1):
        t["gamma+"][m] = float(e["gamma+"][m])
        t["gamma-"][m] = float(e["gamma-"][m])
        for j in range(R + 1):
            t["w+"][m, j] = float(e["w+"][m][j])
            t["w-"][m, j] = float(e["w-"][m][j])
    t["wstar+"] = np.array([float(v) for v in e["wstar+"]])
    t["wstar-"] = np.array([float(v) for v in e["wstar-"]])
    if scheme == "weno-js":
        t["beta_form"] = "B"
        for m in range(R + 1):
            for i in range(R + 1):
                for j in range(R + 1):
                    t["B"][m, i, j] = float(e["B"][m][i][j])
    else:
        t["beta_form"] = "P"
        P, _ = gp_beta_rows_mp(R, _dec(sigma_over_dx), dps)
        for i in range(R + 1):
            for j in range(R + 1):
                t["P"][i, j] = float(P[i][j])
    return t


# ----------------------------------------------------------------------------
# Adaptive-order GP (the paper's Appendix A): GP-AO(R,3) and GP-AO(R',R,3).
# ----------------------------------------------------------------------------
GAMMA_HI = 0.85   # the constants of Eq. (CWENO-lin), "typically" 0.85 (App. A)
GAMMA_LO = 0.85


def cweno_linear_weights(g_hi=GAMMA_HI, g_lo=GAMMA_LO):
    """gamma_1 = gamma_3 = (1 - g_hi)(1 - g_lo)/2, gamma_2 = (1 - g_hi) g_lo (Eq. (CWENO-lin))."""
    return [(1 - g_hi) * (1 - g_lo) / 2, (1 - g_hi) * g_lo, (1 - g_hi) * (1 - g_lo) / 2]


@functools.lru_cache(maxsize=64)
def gp_ao_tables_mp(ell: str, sigma: str, dps: int = DEFAULT_DPS):
    """Tables of GP-AO, in units of dx, for the stencils of radius 3, 2 and the
    three 3-point sub-stencils of the radius-2 stencil (App. A, Eq. (cweno_stencil)).

      'w7+','w7-' : GP weights of the 7-point stencil (nodes -3..3) at x_* = +-1/2
                    (Eq. (q-intrp), length scale ell);
      'w5+','w5-' : the same on the 5-point stencil (nodes -2..2);
      'w3+','w3-' : [m][j] GP weights of the sub-stencils m = 0, 1, 2 (nodes m-2..m);
      'P7','P5','P3' : rows v_i / sqrt(lambda_i) of K_N(sigma), N = 7, 5, 3, so that
                    f^T K_N^-1 f = sum_i (P_i . f)^2 (Eq. (beta-eigen));
      'c7','c5','c3' : N/2 log(2 pi) + 1/2 log det K_N(sigma), the normalisation and
                    complexity terms of the negative log-likelihood (Eq. (log-like)).
    """
    with mp.workdps(dps):
        ellm, sigm = mp.mpf(ell), mp.mpf(sigma)
        out = {}
        for N, R in ((7, 3), (5, 2)):
            nodes = [mp.mpf(j) for j in range(-R, R + 1)]
            K = _kernel_matrix(nodes, ellm)
            for sign, key in ((1, "+"), (-1, "-")):
                out[f"w{N}{key}"] = list(mp.lu_solve(K, _kstar(nodes, mp.mpf(sign) / 2, ellm)))
        nodes5 = [mp.mpf(j) for j in range(-2, 3)]
        for sign, key in ((1, "+"), (-1, "-")):
            xs = mp.mpf(sign) / 2
            out["w3" + key] = [list(mp.lu_solve(_kernel_matrix(nodes5[m:m + 3], ellm), _kstar(nodes5[m:m + 3], xs, ellm)))
                               for m in range(3)]
        for N in (7, 5, 3):
            nodes = [mp.mpf(j) for j in range(N)]
            Ks = _kernel_matrix(nodes, sigm)
            lam, Q = mp.eigsy(Ks)
            out[f"P{N}"] = [[Q[j, i] / mp.sqrt(lam[i]) for j in range(N)] for i in range(N)]
            out[f"c{N}"] = mp.mpf(N) / 2 * mp.log(2 * mp.pi) + sum(mp.log(l) for l in lam) / 2
        return out


def gp_ao_tables(ell_over_dx: float, sigma_over_dx: float, dps: int = DEFAULT_DPS):
    """Float64 arrays of gp_ao_tables_mp, plus the CWENO linear weights and gamma_HI."""
    t = gp_ao_tables_mp(_dec(ell_over_dx), _dec(sigma_over_dx), dps)
    f = lambda v: np.array(v, dtype=float) if not isinstance(v, list) else np.array([[float(x) for x in r] if isinstance(r, list) else float(r) for r in v])  # noqa: E731
    out = {k: f(v) for k, v in t.items() if not k.startswith("c")}
    for N in (7, 5, 3):
        out[f"c{N}"] = float(t[f"c{N}"])
    out["gamma"] = np.array(cweno_linear_weights())
    out["gamma_hi"] = GAMMA_HI
    return out
