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
        Ks = _kernel_matrix(nodes[: R + 1], sigm)
        lam, Q = mp.eigsy(Ks)
        P = []
        for i in range(R + 1):
            P.append([Q[j, i] / mp.sqrt(lam[i]) for j in range(R + 1)])
        out["P"] = P
        out["lambda"] = list(lam)
        return out


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
