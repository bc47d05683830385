"""Reference solutions of radially symmetric Euler problems (test helper).

The explosion data of the paper's Sec. 7 (Eq. (3d-exp)) stay radially
symmetric, so the 3D (or 2D) solution is a function of r = |x| that obeys the
Euler equations with geometric source terms,
    d/dt U + (1/r^a) d/dr (r^a F(U)) = (0, a p / r, 0),   a = ndim - 1,
U = (rho, rho u, E), F = (rho u, rho u^2 + p, u (E + p)). The paper compares its
3D results with such a 1D solution on a fine grid; this module computes one
with an independent, simple method: a finite-volume scheme on cells
[r_{i-1/2}, r_{i+1/2}] with face areas A = r^a and volumes V = r^(a+1)/(a+1)
differences, so that
    V_i dU_i/dt = -(A_{i+1/2} F_{i+1/2} - A_{i-1/2} F_{i-1/2}) + (0, p_i (A_{i+1/2} - A_{i-1/2}), 0)
(the pressure source written this way keeps a uniform state at rest exactly);
minmod-limited linear reconstruction of (rho, u, p), the HLL flux with Davis
wave speeds, SSP-RK2, a mirror image at r = 0 and zero-gradient outflow at
r_max.
"""
from __future__ import annotations

import numpy as np


def _minmod(a, b):
    return np.where(a * b > 0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def _prim(U, g):
    rho = U[0]
    u = U[1] / rho
    p = (g - 1.0) * (U[2] - 0.5 * rho * u * u)
    return rho, u, p


def _flux(rho, u, p, g):
    E = p / (g - 1.0) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, u * (E + p)]), np.array([rho, rho * u, E])


def _rhs(U, a, r_face, vol, g, ng=2):
    rho, u, p = _prim(U, g)
    # ghosts: mirror at r = 0 (u odd), zero gradient at r_max
    def ext(q, odd):
        left = q[:ng][::-1] * (-1.0 if odd else 1.0)
        right = np.repeat(q[-1:], ng)
        return np.concatenate([left, q, right])
    W = [ext(rho, False), ext(u, True), ext(p, False)]
    slopes = [_minmod(w[1:-1] - w[:-2], w[2:] - w[1:-1]) for w in W]
    # states at faces between extended cells j and j+1, j = 1 .. n+2
    L = [w[1:-1][:-1] + 0.5 * s[:-1] for w, s in zip(W, slopes)]
    R = [w[1:-1][1:] - 0.5 * s[1:] for w, s in zip(W, slopes)]
    rL, uL, pL = L
    rR, uR, pR = R
    cL, cR = np.sqrt(g * pL / rL), np.sqrt(g * pR / rR)
    SL = np.minimum(uL - cL, uR - cR)
    SR = np.maximum(uL + cL, uR + cR)
    FL, UL = _flux(rL, uL, pL, g)
    FR, UR = _flux(rR, uR, pR, g)
    hll = (SR * FL - SL * FR + SL * SR * (UR - UL)) / (SR - SL)
    F = np.where(SL >= 0, FL, np.where(SR <= 0, FR, hll))
    n = U.shape[1]
    # face f lies between extended cells f + 1 and f + 2; cell i is extended
    # cell i + ng, so faces r_{-1/2} .. r_{n-1/2} are f = ng - 2 .. ng - 2 + n
    F = F[:, ng - 2: ng - 1 + n]
    A = r_face ** a
    dU = -(A[1:] * F[:, 1:] - A[:-1] * F[:, :-1]) / vol
    dU[1] += p * (A[1:] - A[:-1]) / vol
    return dU


def solve(ndim, left, right, r0, t_final, n=2048, r_max=1.8, g=1.4, cfl=0.4):
    """(r centres, rho, u, p) at t_final for (rho, u, p) = left inside r < r0 and
    right outside, in ndim dimensions (a = ndim - 1)."""
    a = ndim - 1
    r_face = np.linspace(0.0, r_max, n + 1)
    r = 0.5 * (r_face[1:] + r_face[:-1])
    vol = (r_face[1:] ** (a + 1) - r_face[:-1] ** (a + 1)) / (a + 1)
    inside = r < r0
    rho = np.where(inside, left[0], right[0]).astype(float)
    u = np.where(inside, left[1], right[1]).astype(float)
    p = np.where(inside, left[2], right[2]).astype(float)
    _, U = _flux(rho, u, p, g)
    t = 0.0
    dr = r_max / n
    while t < t_final:
        rho, u, p = _prim(U, g)
        dt = cfl * dr / np.max(np.abs(u) + np.sqrt(g * p / rho))
        dt = min(dt, t_final - t)
        U1 = U + dt * _rhs(U, a, r_face, vol, g)
        U = 0.5 * U + 0.5 * (U1 + dt * _rhs(U1, a, r_face, vol, g))
        t += dt
    rho, u, p = _prim(U, g)
    return r, rho, u, p, (U * vol).sum(axis=1)
