"""Whole-run pins of the oracle against exact solutions and the paper's tables.

* Smooth advection has an exact solution (the translated initial data), so the
  measured L1 error must fall at the scheme's design order 2R+1 (Sec. 6: 3, 5, 7
  for R = 1, 2, 3) when ell is held fixed in physical units and the time step is
  reduced as dx^((2R+1)/3) (the paper reduces the time step the same way, Sec. 6.1).
* The paper's Table 1 (Sec. 6.1) and Table 2 (Sec. 6.2) print L1 errors for the
  same problems; the oracle must land close to them. The paper used RK4, this
  scheme uses SSP-RK3 with a reduced step, so the match is not exact: R = 1, 2
  agree within 10 %, R = 3 within 40 %. The paper does not state how its 2D L1
  is normalised; its tabulated values equal 100 x the mean absolute density error
  (checked at every entry run here), which is the reading used.
"""
import math

import numpy as np
import pytest

import inputs
import oracle
from conftest import load_golden


def _run_1d(problem, R, N, ell, gamma, anchor):
    if problem == "sine":
        g, U = inputs.sine_wave_1d(N, gamma)
        _, Ue = inputs.sine_wave_1d(N, gamma, t=1.0)
    else:
        g, U = inputs.gaussian_1d(N, gamma)
        _, Ue = inputs.gaussian_1d(N, gamma, t=1.0)
    dx = g.dx[0]
    s = oracle.OracleSolver(g, R, ell, 3 * dx, gamma)
    smax = s.max_speed(U) * dx
    dx0 = 1.0 / anchor
    dt = 0.4 * dx0 / smax * (dx / dx0) ** ((2 * R + 1) / 3)
    n = math.ceil(1.0 / dt)
    s.run_fixed(U, 1.0 / n, n)
    return float(np.mean(np.abs(U[0] - Ue[0])))


@pytest.mark.parametrize("R,Ns,expect", [(1, (32, 64, 128, 256), 3.0), (2, (32, 64, 128, 256), 5.0),
                                         (3, (32, 64, 128), 7.0)])
def test_convergence_order_fixed_physical_ell(R, Ns, expect):
    errs = [_run_1d("sine", R, N, 0.1, 1.4, 32) for N in Ns]
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(len(errs) - 1)]
    assert orders[-1] == pytest.approx(expect, abs=0.15), (errs, orders)
    assert min(orders) > expect - 0.4


def test_config1_accuracy_against_exact_solution():
    """1D sine wave, N = 128, R = 2, ell = 12 dx, sigma = 3 dx, CFL 0.4 to t = 1."""
    g, U = inputs.sine_wave_1d(128)
    _, Ue = inputs.sine_wave_1d(128, t=1.0)
    s = oracle.OracleSolver(g, 2, 12 * g.dx[0], 3 * g.dx[0], 1.4, 0.4)
    t, n = s.run(U, 1.0)
    assert t == 1.0 and 700 < n < 800
    err = np.mean(np.abs(U[0] - Ue[0]))
    assert 1e-7 < err < 5e-6
    for k in range(3):
        assert abs(U[k].sum() - Ue[k].sum()) <= 1e-13 * np.abs(Ue[k]).sum()


TABLE1 = {int(r[0]): r[1:] for r in load_golden("table1_gaussian_1d.txt")}


@pytest.mark.parametrize("R,N", [(1, 25), (1, 50), (1, 100), (1, 200), (2, 25), (2, 50), (2, 100), (2, 200),
                                 (3, 25), (3, 50), (3, 100)])
def test_paper_table1_gaussian(R, N):
    err = _run_1d("gauss", R, N, 0.1, 5.0 / 3.0, 25)
    paper = TABLE1[N][R - 1]
    tol = 0.10 if R < 3 else 0.40
    assert abs(err / paper - 1.0) < tol, (err, paper)


TABLE2 = {round(r[0], 4): r[1:] for r in load_golden("table2_vortex_2d.txt")}


@pytest.mark.parametrize("R,n", [(1, 50), (2, 50), (3, 50), (2, 100)])
def test_paper_table2_vortex(R, n):
    g, U = inputs.isentropic_vortex_2d(n, lo=0.0, hi=20.0)
    U0 = U.copy()
    dx = g.dx[0]
    s = oracle.OracleSolver(g, R, 1.0, 3 * dx, 1.4)
    dt0 = 0.4 / s.max_speed(U) * (dx / 0.4) ** ((2 * R + 1) / 3 - 1)
    nst = math.ceil(20.0 / dt0)
    s.run_fixed(U, 20.0 / nst, nst)
    err = 100.0 * np.mean(np.abs(U[0] - U0[0]))
    paper = TABLE2[round(dx, 4)][R - 1]
    assert abs(err / paper - 1.0) < 0.05, (err, paper)
