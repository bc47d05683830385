"""Pins of the oracle's adaptive-order GP interpolation (the paper's App. A):
GP-AO(2,3) and GP-AO(3,2,3).

* Tables: the 7- and 5-point GP weights tend to the Lagrange weights as
  ell / dx grows (textbook values), the eigen rows reproduce K_N(sigma)^-1, and
  the normalisation and complexity constants equal N/2 log 2 pi + 1/2 log det
  K_N(sigma) computed with a determinant (not from the eigenvalues).
* The smoothness indicators are the negative log-likelihood of Eq. (log-like)
  with zero mean, recomputed here with numpy's determinant and solve.
* The hybrids: equal indicators return the high-order interpolation exactly
  (Eq. (GP-AO), Eq. (AO-recursive)); a much larger high-order indicator
  returns the GP-CWENO combination, or the lower-order GP-AO; the coefficients
  sum to one; the CWENO linear weights follow Eq. (CWENO-lin).
* Whole runs: a finding of this reading -- the indicators of stencils of
  different size tend to different constants as dx -> 0, so the hybrid weights
  do not tend to their linear values and GP-AO converges at third order on
  smooth data (the GP-CWENO order); a shock tube stays non-oscillatory.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import inputs
import oracle
from oracle.tables import GAMMA_HI, GAMMA_LO, cweno_linear_weights, gp_ao_tables, gp_ao_tables_mp

LAGRANGE7 = np.array([-5, 42, -175, 700, 525, -70, 7]) / 1024
LAGRANGE5 = np.array([3, -20, 90, 60, -5]) / 128
SUB3 = np.array([[3, -10, 15], [-1, 6, 3], [3, 6, -1]]) / 8


def test_cweno_linear_weights():
    g = cweno_linear_weights()
    assert g[0] == g[2] == pytest.approx(0.5 * 0.15 * 0.15)
    assert g[1] == pytest.approx(0.15 * 0.85)
    assert sum(g) == pytest.approx(1 - GAMMA_HI)
    assert GAMMA_HI == GAMMA_LO == 0.85


def test_weights_tend_to_lagrange_weights():
    t = gp_ao_tables(5000.0, 1.8, dps=80)
    assert np.abs(t["w7+"] - LAGRANGE7).max() < 1e-5
    assert np.abs(t["w5+"] - LAGRANGE5).max() < 1e-5
    assert np.abs(t["w3+"] - SUB3).max() < 1e-5
    assert np.abs(t["w7-"] - LAGRANGE7[::-1]).max() < 1e-5


@pytest.mark.parametrize("sigma", [1.5, 1.8, 3.0])
def test_eigen_rows_and_log_det_constants(sigma):
    t = gp_ao_tables_mp("12.0", repr(sigma))
    for N in (7, 5, 3):
        with mp.workdps(60):
            K = mp.matrix(N, N)
            for i in range(N):
                for j in range(N):
                    K[i, j] = mp.exp(-mp.mpf(i - j) ** 2 / (2 * mp.mpf(repr(sigma)) ** 2))
            P = mp.matrix(t[f"P{N}"])
            err = mp.norm(P.T * P * K - mp.eye(N), p=1)
            assert err < mp.mpf(10) ** -35
            c = mp.mpf(N) / 2 * mp.log(2 * mp.pi) + mp.log(mp.det(K)) / 2
            assert abs(c - t[f"c{N}"]) < mp.mpf(10) ** -40


def _neg_log_like(f, sigma):
    N = len(f)
    x = np.arange(N)
    K = np.exp(-(x[:, None] - x[None, :]) ** 2 / (2 * sigma * sigma))
    _, logdet = np.linalg.slogdet(K)
    return N / 2 * math.log(2 * math.pi) + 0.5 * logdet + 0.5 * f @ np.linalg.solve(K, f)


@pytest.mark.parametrize("R", [2, 3])
def test_indicators_are_the_negative_log_likelihood(R):
    sigma = 1.8
    t = gp_ao_tables(12.0, sigma)
    rng = np.random.default_rng(R)
    for _ in range(5):
        f = rng.normal(size=2 * R + 1)
        _, beta = oracle.gp_ao(f, t, 0)
        f5 = f[R - 2: R + 3]
        if R == 3:
            assert beta[0] == pytest.approx(_neg_log_like(f, sigma), rel=1e-9, abs=1e-12)
        assert beta[1] == pytest.approx(_neg_log_like(f5, sigma), rel=1e-9, abs=1e-12)
        for m in range(3):
            assert beta[2 + m] == pytest.approx(_neg_log_like(f5[m:m + 3], sigma), rel=1e-9, abs=1e-12)


GAM = cweno_linear_weights()


def test_hybrid_with_equal_indicators_is_the_high_order_interpolation():
    rng = np.random.default_rng(1)
    for _ in range(10):
        qR, b = rng.normal(), rng.uniform(0.1, 5.0)
        qm = rng.normal(size=3)
        assert oracle.ao_hybrid(qR, b, qm, [b, b, b], GAM, GAMMA_HI) == pytest.approx(qR, abs=1e-14)
        hi, lo = rng.normal(size=2)
        assert oracle.ao_recursive(hi, b, lo, b, GAMMA_HI) == pytest.approx(hi, abs=1e-14)


def test_hybrid_with_a_rough_high_order_stencil_is_the_cweno_combination():
    qm = np.array([0.3, 0.7, -0.2])
    bm = np.array([0.5, 2.0, 1.0])
    w = np.array(GAM) / bm ** 2
    want = float(w @ qm / w.sum())
    assert oracle.ao_hybrid(9.0, 1e9, qm, bm, GAM, GAMMA_HI) == pytest.approx(want, rel=1e-12)
    assert oracle.ao_recursive(9.0, 1e9, 0.25, 1.0, GAMMA_HI) == pytest.approx(0.25, rel=1e-12)


def test_hybrid_coefficients_sum_to_one():
    rng = np.random.default_rng(3)
    for _ in range(20):
        bR = rng.uniform(0.01, 10)
        bm = rng.uniform(0.01, 10, size=3)
        assert oracle.ao_hybrid(1.0, bR, np.ones(3), bm, GAM, GAMMA_HI) == pytest.approx(1.0, abs=1e-13)
        assert oracle.ao_recursive(1.0, bR, 1.0, bm[0], GAMMA_HI) == pytest.approx(1.0, abs=1e-13)


def _sine_error(R, N, sigma):
    g, U = inputs.sine_wave_1d(N)
    _, Ue = inputs.sine_wave_1d(N, t=1.0)
    dx = g.dx[0]
    s = oracle.OracleSolver(g, R, 0.1, sigma * dx, scheme="gp-ao")
    smax = s.max_speed(U) * dx
    dt = 0.4 * (1 / 32) / smax * (dx * 32) ** ((2 * R + 1) / 3)
    n = math.ceil(1.0 / dt)
    s.run_fixed(U, 1.0 / n, n)
    return float(np.mean(np.abs(U[0] - Ue[0])))


@pytest.mark.parametrize("R", [2, 3])
def test_smooth_data_converge_at_third_order(R):
    errs = [_sine_error(R, N, 3.0) for N in (64, 128, 256)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] == pytest.approx(3.0, abs=0.15), (errs, orders)


@pytest.mark.parametrize("R", [2, 3])
def test_shock_tube_stays_non_oscillatory(R):
    g, U = inputs.shock_tube_1d(200)
    dx = g.dx[0]
    t, _ = oracle.OracleSolver(g, R, 12 * dx, 1.8 * dx, scheme="gp-ao").run(U, 0.2)
    assert t == 0.2
    rho, _, p = inputs.cons_to_prim(g, U, 1.4)
    assert rho.max() < 1.0 + 0.015 and rho.min() > 0.125 - 0.015 and p.min() > 0.09
