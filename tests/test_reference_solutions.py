"""Reference solutions used to pin shock problems, and the oracle against them.

* The radial solver (tests/radial_reference.py) in planar geometry reproduces the
  exact Riemann solution of the explosion's two states; in spherical geometry it
  conserves mass and converges under refinement.
* The oracle's 3D explosion (Eq. (3d-exp)) follows the radial reference along
  the x axis and along the diagonal (the paper's Fig. (explosion) comparison).
"""
import numpy as np
import pytest

import inputs
import oracle
import radial_reference as RR
from exact_riemann import sample

IN, OUT = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


@pytest.fixture(scope="module")
def spherical_ref():
    return RR.solve(3, IN, OUT, 0.5, 0.25, n=2048)


def test_planar_radial_solver_matches_the_exact_riemann_solution():
    r, rho, u, p, _ = RR.solve(1, IN, OUT, 0.5, 0.25, n=2048, r_max=1.0)
    ex = sample(IN, OUT, (r - 0.5) / 0.25)
    assert np.mean(np.abs(rho - ex[0])) < 1.5e-3
    assert np.mean(np.abs(p - ex[2])) < 1.5e-3


def test_spherical_radial_solver_conserves_mass_and_converges(spherical_ref):
    r, rho, _, _, tot = spherical_ref
    vol = (np.linspace(0, 1.8, 2049)[1:] ** 3 - np.linspace(0, 1.8, 2049)[:-1] ** 3) / 3
    m0 = float(np.sum(vol * np.where(r < 0.5, IN[0], OUT[0])))
    assert abs(tot[0] - m0) < 1e-12 * m0          # nothing has reached r_max yet
    r2, rho2, _, _, _ = RR.solve(3, IN, OUT, 0.5, 0.25, n=1024)
    assert np.mean(np.abs(np.interp(r2, r, rho) - rho2)) < 5e-3


def profiles(g, rho):
    """Density along the x axis (cells next to it) and along the diagonal, with radii."""
    n = g.n[0]
    dx = g.dx[0]
    x = g.centres(0)
    h = n // 2
    ax, r_ax = rho[h, h, :], np.sqrt(x ** 2 + 2 * (dx / 2) ** 2)
    dg, r_dg = np.array([rho[i, i, i] for i in range(n)]), np.sqrt(3) * np.abs(x)
    return (ax, r_ax), (dg, r_dg)


def test_oracle_explosion_follows_the_radial_reference(spherical_ref):
    r_ref, rho_ref, _, _, _ = spherical_ref
    g, U = inputs.explosion(3, 32)
    dx = g.dx[0]
    t, _ = oracle.OracleSolver(g, 2, 12 * dx, 3 * dx, cfl=0.3).run(U, 0.25)
    assert t == 0.25
    (ax, r_ax), (dg, r_dg) = profiles(g, U[0])
    assert np.mean(np.abs(ax - np.interp(r_ax, r_ref, rho_ref))[r_ax < 0.95]) < 0.04
    assert np.mean(np.abs(dg - np.interp(r_dg, r_ref, rho_ref))[r_dg < 1.0]) < 0.04
