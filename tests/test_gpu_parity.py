"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same
seeded inputs.

Tolerances (relative L1 = sum |gpu - oracle| / sum |oracle| over every field and
cell, the measure the accuracy targets are stated in):
  * float64 path: 1e-12. Both sides evaluate the same formulas in float64; they
    differ only in rounding order (fused multiply-adds, the min-ratio form of the
    nonlinear weights, reciprocal multiplies), i.e. a few ulp per operation, so a
    single right-hand side agrees to ~1e-14 and a few hundred steps to well below
    1e-12.
  * float32 sweep arithmetic: 1e-5. Each right-hand side carries float32
    rounding (~1e-7 relative per operation, amplified by the ill-conditioned
    weights); it enters the float64 state only through dt * L.
Every comparison also holds cell by cell (parity_bounds: 32 eps times the local
flux scale for a right-hand side, that bound integrated over the run for a
state), so a few wrong cells cannot hide inside a grid-wide norm.
"""
import math
import sys

import numpy as np
import pytest

import inputs
import oracle
from parity_bounds import rhs_cell_excess, state_cell_excess

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1808_04960_amd as gw  # noqa: E402


def rel_l1(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def announce(msg):
    print(f"[gpu-parity] {msg}", file=sys.stderr, flush=True)


GRIDS = {
    # several 58-cell runs per pencil with a ragged last run, ragged pencil groups
    1: lambda: inputs.grid1d(200),
    2: lambda: inputs.grid2d(150, 70, (0.0, 0.0), (1.5, 0.7)),
    3: lambda: inputs.grid3d(66, 45, 30, (0.0, 0.0, 0.0), (1.1, 0.75, 0.5)),
}


def flux_bound(g, U, gamma=1.4):
    """sum_i sum_d |F_d(U_i)|_1 / dx_d: the size of the face fluxes a right-hand side
    is differenced from. Rounding of relative size eps in each corrected flux puts
    an error of about 2 eps |F| / dx into the flux difference of a cell, however
    small the difference itself is."""
    rho, vel, p = inputs.cons_to_prim(g, U, gamma)
    E = U[g.nv - 1]
    total = 0.0
    for d in range(g.ndim):
        un = vel[d]
        F = np.abs(rho * un) + np.abs(un * (E + p)) + sum(np.abs(U[1 + e] * un) for e in range(g.ndim)) + np.abs(p)
        total += F.sum() / g.dx[d]
    return float(total)


EPS = {"fp64": 2.0**-53, "fp32": 2.0**-24}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("R", [1, 2, 3])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_rhs_matches_oracle(ndim, R, prec):
    """One right-hand side: sum |L_gpu - L_oracle| <= 16 eps sum_d |F_d| / dx_d, i.e.
    at most 8 ulp-sized errors in each of the two corrected fluxes of a cell (the
    rounding of the GP weights, characteristic projection and HLLC chains)."""
    g = GRIDS[ndim]()
    announce(f"rhs ndim={ndim} R={R} {prec} n={g.n}")
    U = inputs.random_smooth(g, seed=10 * ndim + R)
    dx = g.dx[0]
    ref = oracle.OracleSolver(g, R, 12 * dx, 3 * dx).rhs(U)
    s = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, U0=U)
    got = s.rhs(U)
    err = float(np.abs(got - ref).sum())
    bound = 16 * EPS[prec] * flux_bound(g, U)
    cell = rhs_cell_excess(g, U, got, ref, prec, R)
    announce(f"  abs L1 {err:.3e}  bound {bound:.3e}  rel L1 {rel_l1(got, ref):.3e}  worst cell {cell:.2f}")
    assert err < bound
    assert cell <= 1.0


TINY_SHAPES = [(2,), (3,), (5,), (7,), (13,), (3, 5), (2, 64), (64, 2), (3, 2, 4), (2, 5, 3)]


def tiny_grid(shape, h=1.0 / 64):
    """Square cells of size h on an axis of n cells each (n down to 2)."""
    hi = [n * h for n in shape]
    if len(shape) == 1:
        return inputs.grid1d(shape[0], 0.0, hi[0])
    if len(shape) == 2:
        return inputs.grid2d(shape[0], shape[1], (0.0, 0.0), tuple(hi))
    return inputs.grid3d(*shape, (0.0, 0.0, 0.0), tuple(hi))


@pytest.mark.parametrize("R", [1, 2, 3])
@pytest.mark.parametrize("shape", TINY_SHAPES)
def test_tiny_periodic_axes(shape, R):
    """Periodic axes shorter than a stencil, down to 2 cells: every stencil and
    every 64-cell run wraps the axis more than once (the general modulo of the
    index wrap, runs mostly of unused lanes, x groups with missing columns). One
    right-hand side in both precisions within the bounds of
    test_rhs_matches_oracle, and three steps within the usual 1e-12 / 1e-5 and
    the per-cell state bound."""
    g = tiny_grid(shape)
    dx = g.dx[0]
    U = inputs.random_smooth(g, seed=40 + R)
    announce(f"tiny periodic axes {shape} R={R}")
    o = oracle.OracleSolver(g, R, 12 * dx, 3 * dx)
    ref = o.rhs(U)
    Uo = U.copy()
    t_o, n_o = o.run(Uo, 1e9, max_steps=3)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        s = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, U0=U)
        got = s.rhs(U)
        assert float(np.abs(got - ref).sum()) < 16 * EPS[prec] * flux_bound(g, U)
        assert rhs_cell_excess(g, U, got, ref, prec, R) <= 1.0
        n, t = s.run(1e9, max_steps=3)
        Ug = s.get_state()
        s.close()
        assert n == n_o == 3 and abs(t - t_o) <= (1e-13 if prec == "fp64" else 1e-6) * t_o
        assert rel_l1(Ug, Uo) < tol
        assert state_cell_excess(g, U, Ug, Uo, prec, t, n) <= 1.0


@pytest.mark.parametrize("scale", [1e-20, 1e20])
@pytest.mark.parametrize("R", [1, 2, 3])
def test_rhs_over_the_range_of_the_data(R, scale):
    """Density, momentum and energy scaled together (pressure with them, velocities
    unchanged) by 1e-20 or 1e20: the smoothness indicators move to the eps-dominated
    end (near 1e-40, against eps = 1e-36) or up to about 1e44, where the float64
    sweeps, which form the nonlinear weights over a common denominator, hold
    products of up to three squared indicators (about 1e260). Same bound as the
    unscaled test; the flux sizes scale with the data."""
    g = GRIDS[2]()
    announce(f"rhs scaled by {scale:g} R={R} fp64 n={g.n}")
    U = scale * inputs.random_smooth(g, seed=20 + R)
    dx = g.dx[0]
    ref = oracle.OracleSolver(g, R, 12 * dx, 3 * dx).rhs(U)
    got = gw.Solver(g, R, 12 * dx, 3 * dx, precision="fp64", U0=U).rhs(U)
    err = float(np.abs(got - ref).sum())
    bound = 16 * EPS["fp64"] * flux_bound(g, U)
    cell = rhs_cell_excess(g, U, got, ref, "fp64", R)
    announce(f"  abs L1 {err:.3e}  bound {bound:.3e}  rel L1 {rel_l1(got, ref):.3e}  worst cell {cell:.2f}")
    assert np.isfinite(got).all()
    assert err < bound
    assert cell <= 1.0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_config1_full_run(prec, tol):
    """1D sine wave, N = 128, R = 2, ell = 12 dx, sigma = 3 dx, CFL 0.4, t = 1."""
    announce(f"config1 {prec}")
    g, U = inputs.sine_wave_1d(128)
    dx = g.dx[0]
    o = oracle.OracleSolver(g, 2, 12 * dx, 3 * dx, cfl=0.4)
    Uo = U.copy()
    t_o, n_o = o.run(Uo, 1.0)
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U)
    n, t = s.run(1.0)
    assert n == n_o and t == t_o
    Ug = s.get_state()
    assert rel_l1(Ug, Uo) < tol
    assert state_cell_excess(g, U, Ug, Uo, prec, t, n) <= 1.0
    _, Ue = inputs.sine_wave_1d(128, t=1.0)
    assert np.mean(np.abs(Ug[0] - Ue[0])) < 5e-6


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("R", [1, 2, 3])
def test_vortex_2d_steps(R, prec, tol):
    announce(f"vortex2d R={R} {prec}")
    g, U = inputs.isentropic_vortex_2d(96)
    dx = g.dx[0]
    o = oracle.OracleSolver(g, R, 12 * dx, 3 * dx)
    Uo = U.copy()
    o.run(Uo, 10.0, max_steps=40)
    s = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, U0=U)
    n, t = s.run(10.0, max_steps=40)
    assert n == 40
    Ug = s.get_state()
    assert rel_l1(Ug, Uo) < tol
    assert state_cell_excess(g, U, Ug, Uo, prec, t, n) <= 1.0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_vortex_3d_steps_zero_transverse_field(prec, tol):
    """w = 0 everywhere makes one characteristic field identically zero (beta = 0 on
    every sub-stencil): the float32 weights must stay finite."""
    announce(f"vortex3d {prec}")
    g, U = inputs.isentropic_vortex_3d(24)
    dx = g.dx[0]
    o = oracle.OracleSolver(g, 2, 12 * dx, 3 * dx)
    Uo = U.copy()
    o.run(Uo, 10.0, max_steps=6)
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U)
    n, t = s.run(10.0, max_steps=6)
    Ug = s.get_state()
    assert np.all(np.isfinite(Ug))
    assert rel_l1(Ug, Uo) < tol
    assert state_cell_excess(g, U, Ug, Uo, prec, t, n) <= 1.0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_kelvin_helmholtz_small(prec):
    """Sharp shear-layer data exercise the nonlinear weights (R = 3)."""
    announce(f"KH small {prec}")
    g, U = inputs.kelvin_helmholtz_2d(128, 64)
    dx = g.dx[0]
    o = oracle.OracleSolver(g, 3, 12 * dx, 3 * dx)
    Uo = U.copy()
    o.run(Uo, 1.0, max_steps=20)
    s = gw.Solver(g, 3, 12 * dx, 3 * dx, precision=prec, U0=U)
    n, t = s.run(1.0, max_steps=20)
    Ug = s.get_state()
    assert rel_l1(Ug, Uo) < (1e-12 if prec == "fp64" else 1e-5)
    assert state_cell_excess(g, U, Ug, Uo, prec, t, n) <= 1.0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_free_stream_bitwise_and_conservation(ndim, prec):
    announce(f"free stream ndim={ndim} {prec}")
    g = GRIDS[ndim]()
    U = inputs.uniform_state(g)
    s = gw.Solver(g, 2, 12 * g.dx[0], 3 * g.dx[0], precision=prec, U0=U)
    s.run(1.0, max_steps=5)
    assert np.array_equal(s.get_state(), U)
    U = inputs.random_smooth(g, seed=7)
    s.set_state(U)
    tot0 = s.conserved_sums()
    s.run(1.0, max_steps=25)
    tot1 = s.conserved_sums()
    scale = np.abs(U).reshape(g.nv, -1).sum(axis=1)
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * scale)
    np.testing.assert_allclose(tot0, U.reshape(g.nv, -1).sum(axis=1), rtol=1e-13)


def test_deterministic_repeat():
    announce("determinism")
    g, U = inputs.isentropic_vortex_2d(64)
    outs = []
    for _ in range(2):
        s = gw.Solver(g, 2, 12 * g.dx[0], 3 * g.dx[0], precision="fp32", U0=U)
        s.run(10.0, max_steps=33)
        outs.append(s.get_state())
    assert np.array_equal(outs[0], outs[1])


def test_step_and_run_agree():
    """gpweno_step (eager launches) and gpweno_run (graph replays) give identical states."""
    announce("step vs run")
    g, U = inputs.isentropic_vortex_2d(64)
    a = gw.Solver(g, 2, 12 * g.dx[0], 3 * g.dx[0], U0=U)
    b = gw.Solver(g, 2, 12 * g.dx[0], 3 * g.dx[0], U0=U)
    for _ in range(7):
        a.step(10.0)
    a.synchronize()
    b.run(10.0, max_steps=7)
    assert a.time() == b.time()
    assert np.array_equal(a.get_state(), b.get_state())


def test_nonphysical_state_is_reported():
    announce("non-physical")
    g = inputs.grid2d(64, 64)
    U = inputs.uniform_state(g)
    U[3, 10, 20] = 0.1 * U[3, 10, 20] - 10.0  # negative energy -> negative pressure
    s = gw.Solver(g, 2, 12 * g.dx[0], 3 * g.dx[0], U0=U)
    with pytest.raises(gw.NonPhysicalState):
        s.run(1.0, max_steps=3)


def test_run_that_cannot_advance_time_fails_instead_of_spinning():
    """At t = 1e20 a step of 1 does not change t in float64: the run loop sees a
    replay that moves neither the time nor the end condition and reports it
    (every kernel still runs and exits normally)."""
    announce("stalled run")
    g = inputs.grid1d(64)
    U = inputs.uniform_state(g)    # stays exactly uniform whatever the step
    dx = g.dx[0]
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, fixed_dt=1.0, U0=U)
    s.set_state(U, t=1e20)
    with pytest.raises(gw.GpwenoError) as e:
        s.run(2e20)
    assert e.value.code == gw.ESTATE and "stalled" in str(e.value)


def test_fixed_dt_matches_oracle():
    announce("fixed dt")
    g, U = inputs.sine_wave_1d(64)
    dx = g.dx[0]
    o = oracle.OracleSolver(g, 3, 0.1, 3 * dx)
    Uo = U.copy()
    o.run_fixed(Uo, 1e-3, 50)
    s = gw.Solver(g, 3, 0.1, 3 * dx, fixed_dt=1e-3, U0=U)
    n, t = s.run(1e9, max_steps=50)
    assert n == 50
    Ug = s.get_state()
    assert rel_l1(Ug, Uo) < 1e-12
    assert state_cell_excess(g, U, Ug, Uo, "fp64", t, n) <= 1.0


def test_step_kernels_compose_a_step():
    """The 3*ndim launches exposed one by one (gpweno_step_kernel) form exactly one step."""
    announce("step kernels")
    g, U = inputs.isentropic_vortex_2d(64)
    a = gw.Solver(g, 2, 12 * g.dx[0], 3 * g.dx[0], U0=U)
    b = gw.Solver(g, 2, 12 * g.dx[0], 3 * g.dx[0], U0=U)
    a.step(10.0)
    for k in range(3 * g.ndim):
        a.step_kernel(k)
    a.synchronize()
    b.run(10.0, max_steps=2)
    assert a.time() == b.time()
    assert np.array_equal(a.get_state(), b.get_state())


@pytest.mark.parametrize("R,Ns,expect", [(1, (32, 64, 128, 256), 3.0), (2, (32, 64, 128, 256), 5.0),
                                         (3, (32, 64, 128), 7.0)])
def test_gpu_convergence_orders(R, Ns, expect):
    """The GPU path (float64) reaches the design order 2R+1 on the advected sine
    wave with ell fixed in physical units (0.1) and dt reduced as dx^((2R+1)/3);
    at every resolution it also matches the oracle run."""
    announce(f"convergence R={R}")
    errs = []
    for N in Ns:
        g, U = inputs.sine_wave_1d(N)
        _, Ue = inputs.sine_wave_1d(N, t=1.0)
        dx = g.dx[0]
        o = oracle.OracleSolver(g, R, 0.1, 3 * dx)
        smax = o.max_speed(U) * dx
        dt = 0.4 * (1 / 32) / smax * (dx * 32) ** ((2 * R + 1) / 3)
        n = math.ceil(1.0 / dt)
        s = gw.Solver(g, R, 0.1, 3 * dx, fixed_dt=1.0 / n, U0=U)
        steps, _ = s.run(1e9, max_steps=n)
        assert steps == n
        Ug = s.get_state()
        Uo = U.copy()
        o.run_fixed(Uo, 1.0 / n, n)
        assert rel_l1(Ug, Uo) < 1e-11
        assert state_cell_excess(g, U, Ug, Uo, "fp64", 1.0, n) <= 1.0
        errs.append(float(np.mean(np.abs(Ug[0] - Ue[0]))))
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(len(errs) - 1)]
    announce(f"  L1 {errs} orders {orders}")
    assert orders[-1] == pytest.approx(expect, abs=0.15), (errs, orders)
    assert min(orders) > expect - 0.4
