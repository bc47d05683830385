"""Pins for the oracle's pre-simulation GP tables (Sec. 3.2-3.4, Sec. 4 step 1).

Each table is checked against something other than the code that made it:
  * the large-ell limit, where GP interpolation reduces to polynomial (Lagrange)
    interpolation and the linear weights to the polynomial-WENO ones; both are
    computed here in exact rational arithmetic from their textbook definitions;
  * an exact rational re-solve of the finite-ell systems (fractions, Gaussian
    elimination / normal equations) from the kernel values;
  * the eigen form of the smoothness indicator against the quadratic form
    f^T K_m^{-1} f of Eq. (gp-smooth), evaluated exactly;
  * mirror symmetry between the two prediction points, which the oracle
    computes independently.
"""
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from oracle.tables import gp_tables, gp_tables_mp


def _frac(x, digits=90):
    return Fraction(mp.nstr(x, digits, min_fixed=-1, max_fixed=-1))


def _solve_exact(A, b):
    """Gaussian elimination over the rationals."""
    n = len(A)
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def _lagrange_weights(nodes, x):
    w = []
    for j, xj in enumerate(nodes):
        v = Fraction(1)
        for k, xk in enumerate(nodes):
            if k != j:
                v *= Fraction(x - xk) / Fraction(xj - xk)
        w.append(v)
    return w


@pytest.mark.parametrize("R", [1, 2, 3])
def test_large_ell_limit_is_polynomial_weno(R):
    """As ell/dx -> infinity the GP weights tend to Lagrange interpolation weights
    and gamma to the polynomial-WENO interpolation weights (deviation O((dx/ell)^2))."""
    t = gp_tables_mp(R, "10000.0", "3.0", dps=160)
    half = Fraction(1, 2)
    nodes = list(range(-R, R + 1))
    for sign, key in ((1, "+"), (-1, "-")):
        xs = sign * half
        lag_full = _lagrange_weights(nodes, xs)
        np.testing.assert_allclose([float(v) for v in t["wstar" + key]], [float(v) for v in lag_full], atol=1e-6)
        lag_sub = [_lagrange_weights(nodes[m : m + R + 1], xs) for m in range(R + 1)]
        for m in range(R + 1):
            np.testing.assert_allclose([float(v) for v in t["w" + key][m]], [float(v) for v in lag_sub[m]], atol=1e-6)
        # polynomial case: M gamma = w_* is consistent; forward substitution on rows 0..R
        gam = []
        for r in range(R + 1):
            acc = lag_full[r]
            for n in range(r):
                acc -= gam[n] * lag_sub[n][r - n]
            gam.append(acc / lag_sub[r][0])
        np.testing.assert_allclose([float(v) for v in t["gamma" + key]], [float(v) for v in gam], atol=1e-6)
        assert sum(gam) == 1
    # the textbook fifth-order WENO interpolation weights for R = 2
    if R == 2:
        assert [float(v) for v in gam] == pytest.approx([5 / 16, 10 / 16, 1 / 16])


@pytest.mark.parametrize("R", [1, 2, 3])
def test_weights_match_exact_rational_solve(R):
    """Finite ell = 12 dx: re-solve K w = k_* and the least-squares system exactly."""
    t = gp_tables_mp(R, "12.0", "3.0")
    ell = mp.mpf(12)
    nodes = list(range(-R, R + 1))

    def kern(a, b):
        with mp.workdps(100):
            return _frac(mp.exp(-mp.mpf(a - b) ** 2 / (2 * ell * ell)))

    for sign, key in ((1, "+"), (-1, "-")):
        xs = Fraction(sign, 2)
        K = [[kern(a, b) for b in nodes] for a in nodes]
        with mp.workdps(100):
            ks = [_frac(mp.exp(-(mp.mpf(xs.numerator) / xs.denominator - x) ** 2 / (2 * ell * ell))) for x in nodes]
        w_exact = _solve_exact(K, ks)
        assert max(abs(float(Fraction(mp.nstr(a, 60)) - b)) for a, b in zip(t["wstar" + key], w_exact)) < 1e-40
        subs = []
        for m in range(R + 1):
            idx = list(range(m, m + R + 1))
            Km = [[K[i][j] for j in idx] for i in idx]
            wm = _solve_exact(Km, [ks[i] for i in idx])
            subs.append(wm)
            got = t["w" + key][m]
            assert max(abs(float(Fraction(mp.nstr(a, 60)) - b)) for a, b in zip(got, wm)) < 1e-40
        # least squares through the normal equations, exactly
        M = [[Fraction(0)] * (R + 1) for _ in range(2 * R + 1)]
        for n in range(R + 1):
            for j in range(R + 1):
                M[n + j][n] = subs[n][j]
        MtM = [[sum(M[r][a] * M[r][b] for r in range(2 * R + 1)) for b in range(R + 1)] for a in range(R + 1)]
        Mtw = [sum(M[r][a] * w_exact[r] for r in range(2 * R + 1)) for a in range(R + 1)]
        g_exact = _solve_exact(MtM, Mtw)
        got = t["gamma" + key]
        assert max(abs(float(Fraction(mp.nstr(a, 60)) - b)) for a, b in zip(got, g_exact)) < 1e-35


@pytest.mark.parametrize("R", [1, 2, 3])
@pytest.mark.parametrize("sigma", ["3.0", "1.5"])
def test_beta_eigen_form_equals_quadratic_form(R, sigma):
    """Eq. (beta-eigen) sum_i (P_i . f)^2 must equal f^T K_m^{-1} f (Eq. (gp-smooth))."""
    t = gp_tables_mp(R, "12.0", sigma)
    sig = mp.mpf(sigma)
    with mp.workdps(100):
        Ks = [[_frac(mp.exp(-mp.mpf(a - b) ** 2 / (2 * sig * sig))) for b in range(R + 1)] for a in range(R + 1)]
    rng = np.random.default_rng(R)
    for _ in range(3):
        f = [Fraction(int(v), 7) for v in rng.integers(-20, 20, size=R + 1)]
        x = _solve_exact(Ks, f)
        quad = sum(a * b for a, b in zip(f, x))
        with mp.workdps(60):
            eig = sum((sum(t["P"][i][j] * mp.mpf(f[j].numerator) / f[j].denominator for j in range(R + 1))) ** 2
                      for i in range(R + 1))
        assert abs(float(Fraction(mp.nstr(eig, 60)) - quad)) < 1e-40 * max(1.0, float(quad))
    # eigenvalues are positive (K_m(sigma) is symmetric positive definite)
    assert all(lam > 0 for lam in t["lambda"])


@pytest.mark.parametrize("R", [1, 2, 3])
@pytest.mark.parametrize("ell", [6.0, 12.0, 25.6])
def test_mirror_symmetry_of_the_two_prediction_points(R, ell):
    """x_* = -1/2 is the mirror image of x_* = +1/2: w_m^- = reverse(w_{R-m}^+),
    gamma^- = reverse(gamma^+). The oracle solves both sides independently."""
    t = gp_tables(R, ell, 3.0)
    for m in range(R + 1):
        np.testing.assert_allclose(t["w-"][m, : R + 1], t["w+"][R - m, : R + 1][::-1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(t["gamma-"][: R + 1], t["gamma+"][: R + 1][::-1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(t["wstar-"], t["wstar+"][::-1], rtol=0, atol=1e-15)


def test_weights_do_not_sum_to_one_at_finite_ell():
    """The paper never normalises w or gamma (gamma is a plain least-squares solution,
    Sec. 3.3). At ell = 12 dx their sums differ from 1 by more than roundoff; as
    ell grows they approach the polynomial case, where they sum to 1."""
    t12 = gp_tables(1, 12.0, 3.0)
    assert abs(1.0 - t12["gamma+"].sum()) > 1e-4
    assert abs(1.0 - t12["w+"][0].sum()) > 1e-4
    tbig = gp_tables_mp(1, "10000.0", "3.0", dps=120)
    assert abs(1 - sum(tbig["gamma+"])) < 1e-6
