"""Pins of the oracle's non-periodic boundaries and of shock capturing.

* A reflecting wall is a mirror: the solution on [0, L] with reflecting walls is
  the restriction of the periodic solution on [-L, L] started from the mirror
  extension of the data (density and pressure even, normal velocity odd).
* Reflecting walls conserve mass and energy (the wall fluxes of both vanish,
  also after the high-order correction, whose stencil is mirror-antisymmetric).
* Outflow (zero-gradient) boundaries keep a uniform flow uniform, bitwise.
* Shock tube with the two states of the paper's explosion data (Eq. (3d-exp)):
  the exact Riemann solution (characteristic analysis, tests/exact_riemann.py)
  fixes the star-region plateau, which the scheme must hold to 0.5 %, and the
  density error must fall with resolution.
"""
import math

import numpy as np
import pytest

import inputs
import oracle
from exact_riemann import sample, star_state
from inputs import OUTFLOW, PERIODIC, REFLECT


def _mirror_double_1d(U):
    """Data on [0,1] -> data on [-1,1]: cells reversed on the left half, the
    momentum negated."""
    left = U[:, ::-1].copy()
    left[1] *= -1.0
    return np.concatenate([left, U], axis=1)


@pytest.mark.parametrize("R", [1, 2, 3])
def test_reflecting_wall_is_the_mirror_image_1d(R):
    n = 40
    g = inputs.grid1d(n, 0.0, 1.0, REFLECT)
    U = inputs.random_smooth(g, seed=R)
    g2 = inputs.grid1d(2 * n, -1.0, 1.0)
    U2 = _mirror_double_1d(U)
    dx = g.dx[0]
    a = oracle.OracleSolver(g, R, 12 * dx, 3 * dx)
    b = oracle.OracleSolver(g2, R, 12 * dx, 3 * dx)
    dt = 0.3 / a.max_speed(U)
    a.run_fixed(U, dt, 20)
    b.run_fixed(U2, dt, 20)
    assert np.abs(U2[:, n:] - U).max() < 1e-13 * np.abs(U).max()


def test_reflecting_wall_is_the_mirror_image_2d():
    nx, ny = 36, 24
    g = inputs.grid2d(nx, ny, (0.0, 0.0), (1.0, 1.0), ((REFLECT, REFLECT), (PERIODIC, PERIODIC)))
    U = inputs.random_smooth(g, seed=4)
    g2 = inputs.grid2d(2 * nx, ny, (-1.0, 0.0), (1.0, 1.0))
    left = U[:, :, ::-1].copy()
    left[1] *= -1.0
    U2 = np.ascontiguousarray(np.concatenate([left, U], axis=2))
    dx = g.dx[0]
    a = oracle.OracleSolver(g, 2, 12 * dx, 3 * dx)
    b = oracle.OracleSolver(g2, 2, 12 * dx, 3 * dx)
    dt = 0.3 / a.max_speed(U)
    a.run_fixed(U, dt, 10)
    b.run_fixed(U2, dt, 10)
    assert np.abs(U2[:, :, nx:] - U).max() < 1e-13 * np.abs(U).max()


@pytest.mark.parametrize("R", [1, 2, 3])
def test_reflecting_box_conserves_mass_and_energy(R):
    g = inputs.grid2d(30, 26, (0.0, 0.0), (1.0, 0.9), REFLECT)
    U = inputs.random_smooth(g, seed=10 + R)
    dx = g.dx[0]
    s = oracle.OracleSolver(g, R, 12 * dx, 3 * dx)
    m0, e0 = U[0].sum(), U[3].sum()
    s.run_fixed(U, 0.3 / s.max_speed(U), 15)
    assert abs(U[0].sum() - m0) < 1e-13 * m0
    assert abs(U[3].sum() - e0) < 1e-13 * e0


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_outflow_keeps_a_uniform_flow_bitwise(ndim):
    g = {1: lambda: inputs.grid1d(40, bc=OUTFLOW), 2: lambda: inputs.grid2d(20, 16, bc=OUTFLOW),
         3: lambda: inputs.grid3d(12, 10, 9, bc=OUTFLOW)}[ndim]()
    U = inputs.uniform_state(g)
    U0 = U.copy()
    s = oracle.OracleSolver(g, 2, 0.3, 0.1)
    s.run_fixed(U, 1e-3, 5)
    assert np.array_equal(U, U0)


def test_mixed_boundaries_validate():
    with pytest.raises(ValueError):
        oracle.OracleSolver(inputs.grid1d(40, bc=[(PERIODIC, OUTFLOW)]), 2, 0.3, 0.1)
    with pytest.raises(ValueError):
        oracle.OracleSolver(inputs.grid1d(5, bc=REFLECT), 3, 0.3, 0.5)


LEFT, RIGHT = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


def _tube(n, R=2, lo=0.0, hi=1.0, t=0.2):
    g, U = inputs.shock_tube_1d(n, 0.5, LEFT, RIGHT, lo, hi)
    dx = g.dx[0]
    s = oracle.OracleSolver(g, R, 12 * dx, 3 * dx, cfl=0.4)
    tt, _ = s.run(U, t)
    assert tt == t
    x = g.centres(0)
    rho, vel, p = inputs.cons_to_prim(g, U, 1.4)
    return x, rho, vel[0], p


def test_exact_riemann_solution_of_the_tube():
    """The helper reproduces the tube's star state as published in Riemann-solver
    textbooks (p* = 0.30313, u* = 0.92745) and is continuous across its fans."""
    p, u = star_state(LEFT, RIGHT)
    assert p == pytest.approx(0.30313, abs=1e-5) and u == pytest.approx(0.92745, abs=1e-5)
    v = sample(LEFT, RIGHT, np.array([-math.sqrt(1.4) - 1e-9, -math.sqrt(1.4) + 1e-9]))
    assert np.abs(v[:, 0] - v[:, 1]).max() < 1e-7


@pytest.mark.parametrize("R", [1, 2, 3])
def test_shock_tube_star_plateau(R):
    x, rho, u, p = _tube(400, R)
    ps, us = star_state(LEFT, RIGHT)
    # between the contact (x = 0.5 + 0.2 u*) and the shock (x ~ 0.85), away from both
    band = (x > 0.5 + 0.2 * us + 0.02) & (x < 0.83)
    assert band.sum() > 20
    assert np.median(p[band]) == pytest.approx(ps, rel=5e-3)
    assert np.median(u[band]) == pytest.approx(us, rel=5e-3)
    assert np.abs(p[band] / ps - 1).max() < 0.03


def test_shock_tube_density_error_falls_with_resolution():
    errs = []
    for n in (100, 200, 400):
        x, rho, _, _ = _tube(n)
        exact = sample(LEFT, RIGHT, (x - 0.5) / 0.2)[0]
        errs.append(float(np.mean(np.abs(rho - exact))))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 4e-3 and min(orders) > 0.5, (errs, orders)


def test_outflow_lets_the_waves_leave():
    """The same tube on [0.3, 0.75]: the shock leaves at t ~ 0.14 and the head of
    the rarefaction at t ~ 0.17; the solution inside stays close to the exact one
    (zero-gradient outflow reflects little)."""
    x, rho, _, _ = _tube(180, lo=0.3, hi=0.75)
    exact = sample(LEFT, RIGHT, (x - 0.5) / 0.2)[0]
    xf, rf, _, _ = _tube(400)
    keep = (xf > 0.3) & (xf < 0.75)
    exact_f = sample(LEFT, RIGHT, (xf[keep] - 0.5) / 0.2)[0]
    err_cut = float(np.mean(np.abs(rho - exact)))
    err_full = float(np.mean(np.abs(rf[keep] - exact_f)))
    assert err_cut < 1.5 * err_full, (err_cut, err_full)
