"""Pins for the oracle's per-cell steps and whole-step invariants.

GP-WENO interpolation (Sec. 3.3), the characteristic projection (Sec. 7 intro),
HLLC (Sec. 2 Eq. (riemann_prob), Sec. 7 intro), the flux correction
(Eqs. (numFlux_cor), (FD-ders)) and SSP-RK3 are each checked against closed
forms, special cases and invariants that a plausible mistake would break.
"""
import math

import numpy as np
import pytest

import inputs
import oracle

GAMMA = 1.4


# ---------------------------------------------------------------------------
# GP-WENO interpolation of one variable
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("R", [1, 2, 3])
def test_nonlinear_weights_sum_to_one(R):
    tab = oracle.gp_tables(R, 12.0, 3.0)
    rng = np.random.default_rng(0)
    for _ in range(50):
        f = rng.normal(size=2 * R + 1) * 10 ** rng.uniform(-3, 3)
        _, _, beta, omp, omm = oracle.gp_weno(f, tab)
        assert abs(omp.sum() - 1) < 1e-14 and abs(omm.sum() - 1) < 1e-14
        assert np.all(beta > 0)


@pytest.mark.parametrize("R", [1, 2, 3])
def test_beta_scales_quadratically(R):
    """beta_m(c f) = c^2 beta_m(f), so omega is invariant to scaling the data."""
    tab = oracle.gp_tables(R, 12.0, 3.0)
    f = np.random.default_rng(1).normal(size=2 * R + 1)
    qp, qm, b1, o1, _ = oracle.gp_weno(f, tab)
    qp3, qm3, b3, o3, _ = oracle.gp_weno(3.0 * f, tab)
    np.testing.assert_allclose(b3, 9.0 * b1, rtol=1e-13)
    np.testing.assert_allclose(o3, o1, rtol=1e-12)
    assert qp3 == pytest.approx(3 * qp, rel=1e-13) and qm3 == pytest.approx(3 * qm, rel=1e-13)


@pytest.mark.parametrize("R", [1, 2, 3])
def test_constant_data_uses_linear_weights(R):
    """Equal data on every sub-stencil gives equal beta, so omega = gamma / sum(gamma)
    and the prediction is sum_m (gamma_m/sum gamma) sum_j w_mj times the constant."""
    tab = oracle.gp_tables(R, 12.0, 3.0)
    f = np.full(2 * R + 1, 2.5)
    qp, qm, beta, omp, omm = oracle.gp_weno(f, tab)
    g = tab["gamma+"][: R + 1]
    np.testing.assert_allclose(beta, beta[0], rtol=1e-15)
    np.testing.assert_allclose(omp, g / g.sum(), rtol=1e-14)
    S = sum(g[m] / g.sum() * tab["w+"][m, : R + 1].sum() for m in range(R + 1))
    assert qp == pytest.approx(2.5 * S, rel=1e-14)
    assert qm == pytest.approx(qp, rel=1e-14)  # mirror symmetry of constant data


@pytest.mark.parametrize("R", [1, 2, 3])
def test_mirrored_data_swaps_the_two_predictions(R):
    tab = oracle.gp_tables(R, 12.0, 3.0)
    f = np.random.default_rng(2).normal(size=2 * R + 1)
    qp, qm, *_ = oracle.gp_weno(f, tab)
    qp2, qm2, *_ = oracle.gp_weno(f[::-1].copy(), tab)
    assert qp2 == pytest.approx(qm, rel=1e-13) and qm2 == pytest.approx(qp, rel=1e-13)


@pytest.mark.parametrize("R", [1, 2, 3])
def test_step_data_selects_the_smooth_substencil(R):
    """A jump between cells i and i+1: only sub-stencil m = 0 (nodes i-R..i) is
    smooth, so it gets almost all the weight and q^+ stays near the left value."""
    tab = oracle.gp_tables(R, 12.0, 3.0)
    f = np.array([1.0] * (R + 1) + [0.0] * R)
    qp, qm, beta, omp, omm = oracle.gp_weno(f, tab)
    assert np.argmin(beta) == 0
    assert omp[0] > 0.9
    assert abs(qp - 1.0) < 0.05
    assert abs(qm - 1.0) < 0.05


@pytest.mark.parametrize("R", [1, 2, 3])
def test_smooth_data_interpolates_to_high_order(R):
    """On smooth data the prediction at x_{i+1/2} converges at order 2R+1 when ell is
    held fixed in physical units (large ell/dx reaches the polynomial limit)."""
    errs = []
    for h in (0.02, 0.01):
        tab = oracle.gp_tables(R, 0.5 / h, 3.0)
        x = np.arange(-R, R + 1) * h + 0.3
        f = 1.5 + np.sin(2 * x)
        qp, qm, *_ = oracle.gp_weno(f, tab)
        errs.append(abs(qp - (1.5 + math.sin(2 * (0.3 + h / 2)))))
    order = math.log(errs[0] / errs[1]) / math.log(2)
    assert order > 2 * R + 1 - 0.6


@pytest.mark.parametrize("scheme", ["gp-weno", "weno-gp"])
@pytest.mark.parametrize("R", [1, 2, 3])
def test_weight_ratios_fix_the_exponent_of_eq_weights(R, scheme):
    """Geometric data f_j = r^j make sub-stencil m+1 hold exactly r times the
    data of sub-stencil m. The GP indicator of every sub-stencil is the same
    quadratic form f_m^T K(sigma)^-1 f_m (Eq. (gp-smooth); the sub-stencils are
    translates of one another), so beta_{m+1} = r^2 beta_m, whatever K. With eps
    negligible against beta, Eq. (weights) with p = 2 then gives
    omega_{m+1}/omega_m = (gamma_{m+1}/gamma_m) r^(-2p) = (gamma_{m+1}/gamma_m)
    / r^4 at both points; p = 1 or 3 would give r^-2 or r^-6. (The Jiang-Shu
    forms differ per sub-stencil, so this does not apply to them.)"""
    tab = oracle.gp_tables(R, 12.0, 3.0) if scheme == "gp-weno" else oracle.scheme_tables(scheme, R, 12.0, 3.0)
    for r in (1.5, 2.0, 0.5):
        f = r ** np.arange(2 * R + 1)
        _, _, beta, omp, omm = oracle.gp_weno(f, tab)
        assert beta.min() > 1e-20  # eps = 1e-36 is negligible here
        for m in range(R):
            for om, key in ((omp, "gamma+"), (omm, "gamma-")):
                g = np.asarray(tab[key], dtype=float)
                expect = g[m + 1] / g[m] / r**4
                assert om[m + 1] / om[m] == pytest.approx(expect, rel=1e-12)


@pytest.mark.parametrize("b1", [1e-38, 1e-36, 1e-34, 1e-30])
def test_eps_of_eq_weights_is_1e_minus_36(b1):
    """R = 1 with data (0, 0, a): sub-stencil 0 holds zeros, so beta_0 = 0
    exactly, and beta_1 = a^2 (K^-1)_11 = a^2 / (1 - k^2) for the 2x2 kernel
    matrix of K(sigma) with off-diagonal k = exp(-1/(2 (sigma/dx)^2)) (Eqs.
    (gp-smooth), (kmat)). Eq. (weights) then gives omega_1/omega_0 =
    (gamma_1/gamma_0) (eps/(eps + beta_1))^2, which fixes eps: with a beta_1
    of the order of 1e-36 the ratio moves by orders of magnitude if eps does."""
    import mpmath as mp
    mp.mp.dps = 40
    sig = 3.0
    k = mp.e ** (-1 / (2 * mp.mpf(sig) ** 2))
    a = float(mp.sqrt(mp.mpf(b1) * (1 - k * k)))
    tab = oracle.gp_tables(1, 12.0, sig)
    _, _, beta, omp, omm = oracle.gp_weno(np.array([0.0, 0.0, a]), tab)
    assert beta[0] == 0.0
    bb = mp.mpf(a) ** 2 / (1 - k * k)
    eps = mp.mpf("1e-36")
    for om, key in ((omp, "gamma+"), (omm, "gamma-")):
        g = tab[key]
        expect = mp.mpf(g[1]) / mp.mpf(g[0]) * (eps / (eps + bb)) ** 2
        assert om[1] / om[0] == pytest.approx(float(expect), rel=1e-12)


# ---------------------------------------------------------------------------
# Characteristic projection
# ---------------------------------------------------------------------------
def _prim_jacobian(q, gamma):
    """Jacobian of the 1D Euler equations in primitive variables (rho,u_n,u_t1,u_t2,p)."""
    rho, u, _, _, p = q
    A = np.zeros((5, 5))
    A[0, 0] = u; A[0, 1] = rho
    A[1, 1] = u; A[1, 4] = 1.0 / rho
    A[2, 2] = u
    A[3, 3] = u
    A[4, 1] = gamma * p; A[4, 4] = u
    return A


def test_eigenvectors_diagonalise_the_primitive_jacobian():
    q = np.array([1.3, 0.4, -0.2, 0.7, 0.9])
    L, Rm = oracle.char_vectors(q, GAMMA)
    Rmat = Rm.T  # columns r_k
    np.testing.assert_allclose(L @ Rmat, np.eye(5), atol=1e-14)
    c = math.sqrt(GAMMA * q[4] / q[0])
    D = L @ _prim_jacobian(q, GAMMA) @ Rmat
    np.testing.assert_allclose(D, np.diag([q[1] - c, q[1], q[1], q[1], q[1] + c]), atol=1e-13)


# ---------------------------------------------------------------------------
# HLLC
# ---------------------------------------------------------------------------
def _euler_flux(q, gamma):
    rho, un, t1, t2, p = q
    E = p / (gamma - 1) + 0.5 * rho * (un * un + t1 * t1 + t2 * t2)
    return np.array([rho * un, rho * un * un + p, rho * un * t1, rho * un * t2, un * (E + p)])


def test_hllc_is_consistent():
    q = np.array([0.8, -0.3, 0.5, 0.1, 1.7])
    np.testing.assert_allclose(oracle.hllc(q, q, GAMMA), _euler_flux(q, GAMMA), rtol=1e-14, atol=1e-15)


def test_hllc_supersonic_is_upwind():
    qL = np.array([1.0, 3.0, 0.2, 0.0, 1.0])
    qR = np.array([0.5, 2.8, -0.1, 0.3, 0.7])
    np.testing.assert_allclose(oracle.hllc(qL, qR, GAMMA), _euler_flux(qL, GAMMA), rtol=1e-15)
    qL2 = np.array([1.0, -3.0, 0.2, 0.0, 1.0])
    qR2 = np.array([0.5, -2.8, -0.1, 0.3, 0.7])
    np.testing.assert_allclose(oracle.hllc(qL2, qR2, GAMMA), _euler_flux(qR2, GAMMA), rtol=1e-15)


@pytest.mark.parametrize("u", [0.0, 0.35, -0.35])
def test_hllc_resolves_an_isolated_contact(u):
    """Equal normal velocity and pressure: the exact solution is a contact moving
    at u; HLLC returns the exact upwind flux (this is what HLLC adds to HLL)."""
    qL = np.array([1.0, u, 0.3, -0.2, 0.8])
    qR = np.array([0.25, u, -0.6, 0.5, 0.8])
    F = oracle.hllc(qL, qR, GAMMA)
    up = qL if u >= 0 else qR
    np.testing.assert_allclose(F, _euler_flux(up, GAMMA), rtol=1e-13, atol=1e-15)


def test_hllc_mirror_symmetry():
    qL = np.array([1.1, 0.3, 0.2, -0.4, 1.4])
    qR = np.array([0.6, -0.5, 0.1, 0.2, 0.5])
    F = oracle.hllc(qL, qR, GAMMA)
    flip = np.array([1, -1, 1, 1, 1.0])
    Fm = oracle.hllc(qR * flip, qL * flip, GAMMA)
    np.testing.assert_allclose(Fm, -F * flip, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# High-order flux correction
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", range(0, 8))
def test_flux_correction_exact_to_degree_five(k):
    """F at a face is the cell average of the analytic flux Fhat (Sec. 2, Eq. (prim_F)).
    The corrected flux recovers Fhat exactly for polynomial Fhat of degree <= 5,
    and not beyond."""
    def cell_avg(x):  # average of x^k over [x-1/2, x+1/2] (dx = 1)
        return ((x + 0.5) ** (k + 1) - (x - 0.5) ** (k + 1)) / (k + 1)

    x0 = 0.37
    F5 = np.array([cell_avg(x0 + o) for o in (-2, -1, 0, 1, 2)])
    err = oracle.flux_hat(F5) - x0**k
    if k <= 5:
        assert abs(err) < 1e-13
    else:
        assert abs(err) > 1e-3


@pytest.mark.parametrize("k", range(0, 10))
def test_three_term_flux_correction_exact_to_degree_seven(k):
    """With the sixth-difference term (-5/7168, the next term of the series in
    Eq. (numFlux_cor)) the corrected flux recovers Fhat exactly for polynomial
    Fhat of degree <= 7, and not beyond (same cell-average construction as
    above, seven face fluxes)."""
    def cell_avg(x):
        return ((x + 0.5) ** (k + 1) - (x - 0.5) ** (k + 1)) / (k + 1)

    x0 = 0.37
    F7 = np.array([cell_avg(x0 + o) for o in range(-3, 4)])
    err = oracle.flux_hat(F7) - x0**k
    if k <= 7:
        assert abs(err) < 1e-12
    else:
        assert abs(err) > 1e-4


def test_three_term_correction_in_the_scheme_is_its_sixth_difference():
    """In a whole right-hand side the third term changes only the corrected
    fluxes, by -5/7168 times the sixth difference of the face fluxes. For a
    density wave advected at u = 1 with constant pressure, the face fluxes of a
    sampled sine have a sixth difference of about (2 pi dx)^6 times their
    amplitude, so the two right-hand sides differ by little; across a jump the
    sixth difference is O(1) and they differ by orders of magnitude more."""
    N = 48
    g = inputs.grid1d(N)
    dx = g.dx[0]
    x = (np.arange(N) + 0.5) * dx
    diffs = {}
    for name, rho in (("sine", 1 + 0.2 * np.sin(2 * np.pi * x)), ("sharp", 1 + 0.5 * (x > 0.5))):
        U = inputs.uniform_state(g)
        U[0] = rho
        U[1] = rho * 1.0
        U[2] = 1.0 / 0.4 + 0.5 * rho
        L2 = oracle.OracleSolver(g, 2, 12 * dx, 3 * dx, flux_corr_terms=2).rhs(U)
        L3 = oracle.OracleSolver(g, 2, 12 * dx, 3 * dx, flux_corr_terms=3).rhs(U)
        diffs[name] = float(np.abs(L3 - L2).max())
    # sixth difference of a sampled sine is (2 sin(pi dx))^6 ~ (2 pi dx)^6 times it
    assert 0 < diffs["sine"] < 1e-3
    assert diffs["sharp"] > 100 * diffs["sine"]


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_three_term_correction_keeps_free_stream_and_conservation(ndim):
    g = {1: inputs.grid1d(40), 2: inputs.grid2d(24, 20), 3: inputs.grid3d(12, 10, 9)}[ndim]
    U = inputs.uniform_state(g)
    U0 = U.copy()
    s = oracle.OracleSolver(g, 3, 12 * g.dx[0], 3 * g.dx[0], flux_corr_terms=3)
    s.step(U, 0.01)
    assert np.array_equal(U, U0)
    U = inputs.random_smooth(g, seed=4)
    tot0 = U.reshape(g.nv, -1).sum(axis=1)
    s.run(U, 1.0, max_steps=10)
    tot1 = U.reshape(g.nv, -1).sum(axis=1)
    scale = np.abs(U).reshape(g.nv, -1).sum(axis=1)
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * scale)


# ---------------------------------------------------------------------------
# SSP-RK3
# ---------------------------------------------------------------------------
def test_rk3_amplification_polynomial():
    """On dU/dt = lambda U the three stages give 1 + z + z^2/2 + z^3/6, z = lambda dt."""
    U = np.array([1.0, -0.5, 2.0])
    for z in (0.1, -0.7, -1.9):
        dt = 0.25
        lam = z / dt
        U1 = oracle.rk3_combine(1, U, U, lam * U, dt)
        U2 = oracle.rk3_combine(2, U, U1, lam * U1, dt)
        U3 = oracle.rk3_combine(3, U, U2, lam * U2, dt)
        np.testing.assert_allclose(U3, U * (1 + z + z * z / 2 + z**3 / 6), rtol=1e-14)


# ---------------------------------------------------------------------------
# Whole-step invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("R", [1, 2, 3])
def test_free_stream_is_preserved_bitwise(ndim, R):
    g = {1: inputs.grid1d(16), 2: inputs.grid2d(12, 10), 3: inputs.grid3d(10, 9, 8)}[ndim]
    U = inputs.uniform_state(g)
    U0 = U.copy()
    s = oracle.OracleSolver(g, R, 12 * g.dx[0], 3 * g.dx[0])
    L = s.rhs(U)
    assert np.all(L == 0.0)
    s.step(U, 0.01)
    assert np.array_equal(U, U0)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_conservation_to_roundoff(ndim):
    g = {1: inputs.grid1d(64), 2: inputs.grid2d(24, 20), 3: inputs.grid3d(12, 10, 8)}[ndim]
    U = inputs.random_smooth(g, seed=3)
    s = oracle.OracleSolver(g, 2, 12 * g.dx[0], 3 * g.dx[0])
    tot0 = U.reshape(g.nv, -1).sum(axis=1)
    s.run(U, 1.0, max_steps=20)
    tot1 = U.reshape(g.nv, -1).sum(axis=1)
    scale = np.abs(U).reshape(g.nv, -1).sum(axis=1)
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * scale)


@pytest.mark.parametrize("ndim,axis", [(1, 0), (2, 0), (2, 1), (3, 2)])
def test_mirror_image_gives_mirror_solution(ndim, axis):
    g = {1: inputs.grid1d(40), 2: inputs.grid2d(20, 18), 3: inputs.grid3d(10, 9, 12)}[ndim]
    U = inputs.random_smooth(g, seed=5)
    Um = inputs.mirror(g, U, axis)
    s = oracle.OracleSolver(g, 2, 12 * g.dx[0], 3 * g.dx[0])
    s.step(U, 2e-3)
    s.step(Um, 2e-3)
    np.testing.assert_allclose(inputs.mirror(g, Um, axis), U, rtol=1e-13, atol=1e-13)


def test_2d_reduces_to_1d_along_either_axis():
    """A 2D state that varies only along x (v = 0) evolves like the 1D problem on every
    row; the same state rotated to vary along y evolves like its transpose."""
    n, m = 32, 6
    g1, U1 = inputs.sine_wave_1d(n)
    g2 = inputs.grid2d(n, m, (0.0, 0.0), (1.0, m / n))
    rho, vel, p = inputs.cons_to_prim(g1, U1, GAMMA)
    U2 = inputs.prim_to_cons(g2, np.tile(rho, (m, 1)), [np.tile(vel[0], (m, 1)), np.zeros((m, n))],
                             np.tile(p, (m, 1)), GAMMA)
    gT = inputs.grid2d(m, n, (0.0, 0.0), (m / n, 1.0))
    UT = np.ascontiguousarray(np.stack([U2[0].T, U2[2].T, U2[1].T, U2[3].T]))
    ell, sig = 12 / n, 3 / n
    s1 = oracle.OracleSolver(g1, 2, ell, sig)
    s2 = oracle.OracleSolver(g2, 2, ell, sig)
    sT = oracle.OracleSolver(gT, 2, ell, sig)
    for _ in range(5):
        s1.step(U1, 4e-3)
        s2.step(U2, 4e-3)
        sT.step(UT, 4e-3)
    for j in range(m):
        np.testing.assert_allclose(U2[0, j], U1[0], rtol=1e-14)
        np.testing.assert_allclose(U2[1, j], U1[1], rtol=1e-14)
        np.testing.assert_allclose(U2[3, j], U1[2], rtol=1e-14)
    assert np.all(U2[2] == 0.0)
    np.testing.assert_allclose(UT[0].T, U2[0], rtol=1e-14)
    np.testing.assert_allclose(UT[2].T, U2[1], rtol=1e-14)


def test_cfl_time_step_reading():
    """dt = CFL / max_i sum_d (|u_d| + c)/dx_d, clipped to t_final."""
    g = inputs.grid2d(8, 6, (0, 0), (1.0, 2.0))
    U = inputs.uniform_state(g, rho=1.2, vel=(0.5, -0.25), p=0.8)
    s = oracle.OracleSolver(g, 2, 12 * g.dx[0], 3 * g.dx[0], cfl=0.4)
    c = math.sqrt(GAMMA * 0.8 / 1.2)
    speed = (0.5 + c) / g.dx[0] + (0.25 + c) / g.dx[1]
    assert s.max_speed(U) == pytest.approx(speed, rel=1e-15)
    assert s.dt(U, 0.0, 1.0) == pytest.approx(0.4 / speed, rel=1e-15)
    assert s.dt(U, 1.0 - 1e-4, 1.0) == pytest.approx(1e-4, rel=1e-9)
