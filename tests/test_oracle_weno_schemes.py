"""Pins of the oracle's comparison schemes (Sec. 6.2, Table (weno-vortex)):
polynomial WENO interpolation of point values with Jiang-Shu smoothness
indicators (WENO-JS) or with the GP indicators of Eq. (beta-eigen) (WENO-GP).

* The exact rational tables equal the textbook values: Lagrange weights of the
  sub-stencils and the whole stencil at x = +-1/2, the linear weights of WENO
  interpolation, and for R = 2 the Jiang-Shu indicators
  13/12 (second difference)^2 + 1/4 (first-derivative stencil)^2, for R = 1 the
  squared first difference.
* Polynomial weights reproduce quadratic data exactly whatever the nonlinear
  weights are; linear data gives equal indicators and hence the linear weights.
* Jumps: the sub-stencils that cross a discontinuity get negligible weight.
* Whole runs: WENO-JS with R = 2 converges at order 5. WENO-JS with R = 1 falls to
  order 2 on a sine wave (the known loss of the three-point Jiang-Shu weights at
  critical points), while the same interpolation with GP indicators (WENO-GP)
  keeps orders 3 / 5 / 7.
* The paper's Table (weno-vortex), WENO-GP column, within 5 %.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import inputs
import oracle
from conftest import load_golden
from oracle.tables import poly_weno_tables_exact, scheme_tables

TEXTBOOK = {
    1: {"wstar+": [Fr(-1, 8), Fr(6, 8), Fr(3, 8)], "gamma+": [Fr(1, 4), Fr(3, 4)],
        "w+": [[Fr(-1, 2), Fr(3, 2)], [Fr(1, 2), Fr(1, 2)]]},
    2: {"wstar+": [Fr(3, 128), Fr(-20, 128), Fr(90, 128), Fr(60, 128), Fr(-5, 128)],
        "gamma+": [Fr(1, 16), Fr(10, 16), Fr(5, 16)],
        "w+": [[Fr(3, 8), Fr(-10, 8), Fr(15, 8)], [Fr(-1, 8), Fr(6, 8), Fr(3, 8)], [Fr(3, 8), Fr(6, 8), Fr(-1, 8)]]},
    3: {"wstar+": [Fr(k, 1024) for k in (-5, 42, -175, 700, 525, -70, 7)],
        "gamma+": [Fr(1, 64), Fr(21, 64), Fr(35, 64), Fr(7, 64)]},
}


@pytest.mark.parametrize("R", [1, 2, 3])
def test_polynomial_tables_equal_textbook_values(R):
    t = poly_weno_tables_exact(R)
    for key, want in TEXTBOOK[R].items():
        assert t[key] == want, key
    # x_* = -1/2 is the mirror image
    assert t["wstar-"] == t["wstar+"][::-1]
    assert t["gamma-"] == t["gamma+"][::-1]
    for m in range(R + 1):
        assert t["w-"][m] == t["w+"][R - m][::-1]


def _quadform(f):
    return np.outer(f, f)


def test_jiang_shu_forms_equal_textbook_formulas():
    B = poly_weno_tables_exact(2)["B"]
    d2 = np.array([1, -2, 1])
    first = [np.array([1, -4, 3]), np.array([1, 0, -1]), np.array([3, -4, 1])]
    for m in range(3):
        want = Fr(13, 12) * _quadform(d2) + Fr(1, 4) * _quadform(first[m])
        assert [[Fr(x) for x in row] for row in want] == B[m]
    B1 = poly_weno_tables_exact(1)["B"]
    for m in range(2):
        assert B1[m] == [[1, -1], [-1, 1]]


def _js_beta_textbook(f):
    a, b, c, d, e = f
    return np.array([13 / 12 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2,
                     13 / 12 * (b - 2 * c + d) ** 2 + 0.25 * (b - d) ** 2,
                     13 / 12 * (c - 2 * d + e) ** 2 + 0.25 * (3 * c - 4 * d + e) ** 2])


def test_c_oracle_js_beta_and_weights_on_random_data():
    tab = scheme_tables("weno-js", 2, 12.0, 3.0)
    rng = np.random.default_rng(11)
    for _ in range(50):
        f = rng.normal(size=5)
        qp, qm, beta, omp, omm = oracle.gp_weno(f, tab)
        want = _js_beta_textbook(f)
        np.testing.assert_allclose(beta, want, rtol=1e-13)
        wt = np.array([1 / 16, 10 / 16, 5 / 16]) / (1e-36 + want) ** 2
        np.testing.assert_allclose(omp, wt / wt.sum(), rtol=1e-12)
        sub = [3 / 8 * f[0] - 10 / 8 * f[1] + 15 / 8 * f[2], -1 / 8 * f[1] + 6 / 8 * f[2] + 3 / 8 * f[3],
               3 / 8 * f[2] + 6 / 8 * f[3] - 1 / 8 * f[4]]
        assert qp == pytest.approx(float(np.dot(omp, sub)), rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("scheme,R", [("weno-js", 1), ("weno-js", 2), ("weno-gp", 1), ("weno-gp", 2),
                                      ("weno-gp", 3)])
def test_polynomial_interpolation_is_exact_for_quadratics(scheme, R):
    tab = scheme_tables(scheme, R, 12.0, 3.0)
    rng = np.random.default_rng(R)
    x = np.arange(-R, R + 1, dtype=np.float64)
    for _ in range(20):
        a, b, c = rng.normal(size=3)
        f = a + b * x + (c * x * x if R > 1 else 0.0)
        qp, qm, _, _, _ = oracle.gp_weno(f, tab)
        p = lambda s: a + b * s + (c * s * s if R > 1 else 0.0)  # noqa: E731
        assert qp == pytest.approx(p(0.5), abs=1e-13)
        assert qm == pytest.approx(p(-0.5), abs=1e-13)


@pytest.mark.parametrize("R", [1, 2])
def test_linear_data_gives_linear_weights(R):
    tab = scheme_tables("weno-js", R, 12.0, 3.0)
    f = 0.3 + 0.7 * np.arange(-R, R + 1)
    qp, qm, beta, omp, omm = oracle.gp_weno(f, tab)
    assert np.allclose(beta, beta[0], rtol=1e-14)
    g = np.array([float(v) for v in poly_weno_tables_exact(R)["gamma+"]])
    np.testing.assert_allclose(omp, g / g.sum(), rtol=1e-14)
    assert qp == pytest.approx(0.3 + 0.35, abs=1e-14)


def test_jump_gets_negligible_weight():
    # jump between nodes 0 and +1: only sub-stencil 0 (nodes -2..0) is smooth;
    # constant data there has a zero Jiang-Shu indicator
    tab = scheme_tables("weno-js", 2, 12.0, 3.0)
    qp, qm, beta, omp, omm = oracle.gp_weno(np.array([1.0, 1.0, 1.0, 0.0, 0.0]), tab)
    assert beta[0] < 1e-14
    assert omp[1] + omp[2] < 1e-25 and omm[1] + omm[2] < 1e-25
    assert qp == pytest.approx(1.0, abs=1e-14) and qm == pytest.approx(1.0, abs=1e-14)


def test_jump_with_gp_indicators():
    # the zero-mean GP indicator of constant data is not zero (f^T K^-1 f > 0), so
    # the smooth sub-stencil dominates without taking all the weight; the weights
    # are those of GP-WENO on the same data, up to the different linear weights
    f = np.array([1.0, 1.0, 1.0, 0.0, 0.0])
    _, _, b_gp, om_gp, _ = oracle.gp_weno(f, scheme_tables("gp-weno", 2, 12.0, 3.0))
    _, _, b_wg, om_wg, _ = oracle.gp_weno(f, scheme_tables("weno-gp", 2, 12.0, 3.0))
    np.testing.assert_array_equal(b_gp, b_wg)
    assert om_wg[0] > 0.98 and om_wg[2] < 0.01
    assert abs(om_wg - om_gp).max() < 1e-3


def _sine_error(scheme, R, N):
    g, U = inputs.sine_wave_1d(N)
    _, Ue = inputs.sine_wave_1d(N, t=1.0)
    dx = g.dx[0]
    s = oracle.OracleSolver(g, R, 0.1, 3 * dx, 1.4, scheme=scheme)
    smax = s.max_speed(U) * dx
    dx0 = 1.0 / 32
    dt = 0.4 * dx0 / smax * (dx / dx0) ** ((2 * R + 1) / 3)
    n = math.ceil(1.0 / dt)
    s.run_fixed(U, 1.0 / n, n)
    return float(np.mean(np.abs(U[0] - Ue[0])))


@pytest.mark.parametrize("scheme,R,Ns,expect", [
    ("weno-js", 2, (32, 64, 128, 256), 5.0),
    ("weno-js", 1, (64, 128, 256), 2.0),
    ("weno-gp", 1, (64, 128, 256), 3.0),
    ("weno-gp", 2, (64, 128, 256), 5.0),
    ("weno-gp", 3, (32, 64, 128), 7.0),
])
def test_convergence_orders(scheme, R, Ns, expect):
    errs = [_sine_error(scheme, R, N) for N in Ns]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] == pytest.approx(expect, abs=0.15), (errs, orders)


TABLE3 = {round(r[0], 4): r[1:] for r in load_golden("table3_weno_vortex_2d.txt")}


@pytest.mark.parametrize("n", [50, 100])
def test_paper_table3_weno_gp_column(n):
    g, U = inputs.isentropic_vortex_2d(n, lo=0.0, hi=20.0)
    U0 = U.copy()
    dx = g.dx[0]
    s = oracle.OracleSolver(g, 2, 1.0, 3 * dx, 1.4, scheme="weno-gp")
    dt0 = 0.4 / s.max_speed(U) * (dx / 0.4) ** (5 / 3 - 1)
    nst = math.ceil(20.0 / dt0)
    s.run_fixed(U, 20.0 / nst, nst)
    err = 100.0 * np.mean(np.abs(U[0] - U0[0]))
    paper = TABLE3[round(dx, 4)][1]
    assert abs(err / paper - 1.0) < 0.05, (err, paper)
