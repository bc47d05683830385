"""Exact solution of the 1D Riemann problem of the Euler equations for an ideal
gas, used to pin shock-capturing runs (test helper; written from the
characteristic analysis of the Riemann problem: the star-region pressure is the
root of f_L(p) + f_R(p) + u_R - u_L = 0, with the shock (Rankine-Hugoniot) and
rarefaction (isentropic) branches of f_K, and the self-similar solution is
sampled along x/t)."""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rho, pK, g):
    c = math.sqrt(g * pK / rho)
    if p > pK:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        return (p - pK) * math.sqrt(A / (p + B))
    return 2.0 * c / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(left, right, g=1.4):
    """(p*, u*) of the Riemann problem with left/right = (rho, u, p)."""
    rL, uL, pL = left
    rR, uR, pR = right
    f = lambda p: _fK(p, rL, pL, g) + _fK(p, rR, pR, g) + uR - uL  # noqa: E731
    lo, hi = 1e-14, max(pL, pR)
    while f(hi) < 0:
        hi *= 2.0
    for _ in range(200):  # bisection: f is increasing in p
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    p = 0.5 * (lo + hi)
    u = 0.5 * (uL + uR) + 0.5 * (_fK(p, rR, pR, g) - _fK(p, rL, pL, g))
    return p, u


def sample(left, right, xi, g=1.4):
    """(rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    rL, uL, pL = left
    rR, uR, pR = right
    ps, us = star_state(left, right, g)
    cL, cR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)
    gm = (g - 1.0) / (g + 1.0)
    out = np.zeros((3, len(xi)))
    for k, s in enumerate(np.asarray(xi, dtype=float)):
        if s <= us:  # left of the contact
            if ps > pL:
                SL = uL - cL * math.sqrt((g + 1.0) / (2.0 * g) * ps / pL + (g - 1.0) / (2.0 * g))
                if s <= SL:
                    v = (rL, uL, pL)
                else:
                    v = (rL * (ps / pL + gm) / (gm * ps / pL + 1.0), us, ps)
            else:
                cs = cL * (ps / pL) ** ((g - 1.0) / (2.0 * g))
                if s <= uL - cL:
                    v = (rL, uL, pL)
                elif s >= us - cs:
                    v = (rL * (ps / pL) ** (1.0 / g), us, ps)
                else:
                    fac = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * cL) * (uL - s)
                    v = (rL * fac ** (2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (cL + (g - 1.0) / 2.0 * uL + s),
                         pL * fac ** (2.0 * g / (g - 1.0)))
        else:  # right of the contact
            if ps > pR:
                SR = uR + cR * math.sqrt((g + 1.0) / (2.0 * g) * ps / pR + (g - 1.0) / (2.0 * g))
                if s >= SR:
                    v = (rR, uR, pR)
                else:
                    v = (rR * (ps / pR + gm) / (gm * ps / pR + 1.0), us, ps)
            else:
                cs = cR * (ps / pR) ** ((g - 1.0) / (2.0 * g))
                if s >= uR + cR:
                    v = (rR, uR, pR)
                elif s <= us + cs:
                    v = (rR * (ps / pR) ** (1.0 / g), us, ps)
                else:
                    fac = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * cR) * (uR - s)
                    v = (rR * fac ** (2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (-cR + (g - 1.0) / 2.0 * uR + s),
                         pR * fac ** (2.0 * g / (g - 1.0)))
        out[:, k] = v
    return out
