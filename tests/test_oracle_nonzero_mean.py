"""Pins of the non-zero-mean GP smoothness indicator (Sec. 7, scalar advection):
beta_m computed from f_m - f_i, f_i the centre cell's value.

* It is the quadratic form (f_m - f_i)^T K_m(sigma)^{-1} (f_m - f_i), evaluated
  here in high precision from the kernel matrix (not from the oracle's tables).
* It vanishes on constant data, and is unchanged when a constant is added.
* At a jump the smooth sub-stencil, whose data equal the centre value, gets all
  the weight.
* The paper's observation: zero-mean GP-R2 leaves Gibbs oscillations at the
  edges of an advected square pulse, the non-zero mean removes them.
"""

import mpmath as mp
import numpy as np
import pytest

import inputs
import oracle
from oracle.tables import gp_tables


def _beta_exact(f_sub, centre, sigma):
    """(f - c)^T K^{-1} (f - c) with K_jk = exp(-(j-k)^2 / (2 sigma^2)), 50 digits."""
    n = len(f_sub)
    with mp.workdps(50):
        K = mp.matrix(n, n)
        for j in range(n):
            for k in range(n):
                K[j, k] = mp.exp(-mp.mpf(j - k) ** 2 / (2 * mp.mpf(sigma) ** 2))
        d = mp.matrix([mp.mpf(v) - mp.mpf(centre) for v in f_sub])
        x = mp.lu_solve(K, d)
        return float(sum(d[i] * x[i] for i in range(n)))


@pytest.mark.parametrize("R", [1, 2, 3])
def test_indicator_is_the_centred_quadratic_form(R):
    tab = gp_tables(R, 12.0, 3.0)
    rng = np.random.default_rng(40 + R)
    for _ in range(5):
        f = rng.normal(size=2 * R + 1)
        _, _, beta, _, _ = oracle.gp_weno(f, tab, nonzero_mean=True)
        for m in range(R + 1):
            want = _beta_exact(list(f[m: m + R + 1]), f[R], 3.0)
            assert beta[m] == pytest.approx(want, rel=1e-11, abs=1e-14)


@pytest.mark.parametrize("R", [1, 2, 3])
def test_constants_do_not_change_the_indicator(R):
    tab = gp_tables(R, 12.0, 3.0)
    _, _, beta0, _, _ = oracle.gp_weno(np.full(2 * R + 1, 3.7), tab, nonzero_mean=True)
    assert not beta0.any()
    f = np.random.default_rng(R).normal(size=2 * R + 1)
    _, _, b1, _, _ = oracle.gp_weno(f, tab, nonzero_mean=True)
    _, _, b2, _, _ = oracle.gp_weno(f + 0.75, tab, nonzero_mean=True)
    np.testing.assert_allclose(b2, b1, rtol=1e-12)


def test_jump_is_avoided_completely():
    tab = gp_tables(2, 12.0, 3.0)
    qp, qm, beta, omp, omm = oracle.gp_weno(np.array([1.0, 1.0, 1.0, 0.0, 0.0]), tab, nonzero_mean=True)
    assert beta[0] == 0.0
    assert omp[1] + omp[2] < 1e-60 and omm[1] + omm[2] < 1e-60


def _square_pulse(nonzero_mean, n=200):
    g = inputs.grid1d(n)
    x = g.centres(0)
    rho = 1.0 + ((x > 0.3) & (x < 0.6)).astype(float)
    U = inputs.prim_to_cons(g, rho, [np.ones(n)], np.ones(n), 1.4)
    dx = g.dx[0]
    s = oracle.OracleSolver(g, 2, 12 * dx, 3 * dx, nonzero_mean=nonzero_mean)
    s.run(U, 1.0)   # one period
    return U[0]


def test_nonzero_mean_removes_the_gibbs_oscillations_of_a_square_pulse():
    zero = _square_pulse(False)
    nonzero = _square_pulse(True)
    over_zero = max(zero.max() - 2.0, 1.0 - zero.min())
    over_nonzero = max(nonzero.max() - 2.0, 1.0 - nonzero.min())
    assert over_zero > 0.03          # a visible overshoot (7 % of the jump)
    assert over_nonzero < 1e-3       # essentially none
