"""Per-cell parity bounds of the GPU path against the oracle (test helper).

A relative L1 over the whole grid can hide a few wrong cells (a seam, a ragged
last run, a transposed output row). These bounds hold cell by cell.

Right-hand side. L_i = -(fhat_{i+1/2} - fhat_{i-1/2})/dx per direction, and
each corrected flux is a chain of a few dozen dependent operations (projection
of 2R+1 values, weights, back-projection, HLLC, the correction over 5 or 7
face fluxes) on values of the size of the face fluxes in its stencil. Both
sides round differently (fused multiply-adds, reciprocals, evaluation order),
so a corrected flux may differ by some ulps of the largest face flux within
reach. The L1 tests allow 8 ulp per corrected flux on average; a single cell
is allowed twice that, 16 ulp per corrected flux, i.e.
    |L_gpu - L_oracle|_{k,i} <= 32 eps s_i,
    s_i = sum_d max_{|j - i|_d <= R + 1 + NC} |F_d(U_j)|_1 / dx_d,
with eps the unit roundoff of the sweep arithmetic and the max over the cells
whose fluxes reach cell i along axis d.

States after a run to time t. Each stage adds dt L to a float64 state; the
SSP-RK3 weights of the three stages' dt L sum to one per step, so the
right-hand-side bound integrates to 32 eps t S over the run, S = max_i s_i at
reach 0 over the initial and final states (the scheme is stable, so earlier
errors are not amplified), plus the float64 rounding of the stage
combinations, a few ulp of |U| per step on each side:
    |U_gpu - U_oracle|_{k,i} <= 32 eps t S + 4 n eps64 max|U_k|.

Conserved totals of a periodic run. The flux differences telescope, so the
exact totals do not change; the float64 totals before and after n steps differ
by the rounding of the per-cell stage updates (8 n eps64 sum|U_k|) and by the
rounding of the two reductions that form them (conserved_totals_bound).
"""
import numpy as np

import inputs

EPS = {"fp64": 2.0**-53, "fp32": 2.0**-24}


def face_flux_sizes(g, U, gamma=1.4):
    """Per axis d and cell: sum over components of |F_d(U_i)|, divided by dx_d."""
    rho, vel, p = inputs.cons_to_prim(g, U, gamma)
    E = U[g.nv - 1]
    out = []
    for d in range(g.ndim):
        un = vel[d]
        F = np.abs(rho * un) + np.abs(un * (E + p)) + sum(np.abs(U[1 + e] * un) for e in range(g.ndim)) + np.abs(p)
        out.append(F / g.dx[d])
    return out


def local_flux_scale(g, U, reach, gamma=1.4):
    """s_i: per axis, the largest flux size within `reach` cells along that axis
    (periodic neighbours; at a non-periodic side the wrap only enlarges the
    scale), summed over axes."""
    sizes = face_flux_sizes(g, U, gamma)
    tot = np.zeros(g.shape)
    for d in range(g.ndim):
        ax = g.ndim - 1 - d
        m = sizes[d].copy()
        for o in range(1, reach + 1):
            m = np.maximum(m, np.maximum(np.roll(sizes[d], o, axis=ax), np.roll(sizes[d], -o, axis=ax)))
        tot += m
    return tot


def rhs_cell_excess(g, U, got, ref, prec, R, nc=2, gamma=1.4):
    """Largest ratio |L_gpu - L_oracle| / (32 eps s_i) over cells and fields
    (<= 1 passes)."""
    s = local_flux_scale(g, U, R + 1 + nc, gamma)
    return float((np.abs(got - ref) / (32 * EPS[prec] * s[None])).max())


def state_cell_excess(g, U0, got, ref, prec, t, nsteps, gamma=1.4):
    """Largest ratio |U_gpu - U_oracle| / bound over cells and fields after a run
    of nsteps steps to time t from U0 (<= 1 passes)."""
    S = max(float(local_flux_scale(g, U0, 0, gamma).max()), float(local_flux_scale(g, ref, 0, gamma).max()))
    umax = np.abs(ref).reshape(g.nv, -1).max(axis=1)
    bound = 32 * EPS[prec] * t * S + 4 * nsteps * EPS["fp64"] * umax
    err = np.abs(got - ref).reshape(g.nv, -1).max(axis=1)
    return float((err / bound).max())


def sum_rounding_depth(ncell):
    """Additions a term passes through in the library's float64 totals: each
    thread of 1024 x 256 adds its cells at a fixed stride (ceil(ncell / 262144)
    terms), a tree of 8 levels joins a block's 256 threads, and one thread adds
    the 1024 block partials in order. The computed sum then differs from the
    exact one by at most that depth times eps64 sum|x| (to first order)."""
    m = -(-int(ncell) // (1024 * 256))
    return (m - 1) + 8 + 1023


def conserved_totals_bound(ncell, nsteps, abs_totals):
    """Largest change of the float64 conserved totals over nsteps steps of a
    periodic run: 8 eps64 sum|U_k| per step for the stage updates, plus the
    rounding of the two reductions. A field that is zero everywhere (bound 0)
    must stay exactly zero."""
    return (8 * nsteps + 2 * sum_rounding_depth(ncell)) * EPS["fp64"] * np.asarray(abs_totals)
