"""Non-periodic boundaries and shock capturing on the GPU, against the oracle.

* Right-hand sides with outflow and reflecting sides (mixed per axis) agree with
  the oracle within the rounding bound of the flux difference.
* Shock tube (the two states of the paper's explosion data, Eq. (3d-exp)) and the
  3D explosion itself: whole runs agree with the oracle (1e-12 fp64, 1e-5 fp32).
* A reflecting wall equals the periodic mirror-doubled problem; a reflecting box
  conserves mass and energy; outflow keeps uniform flow bitwise.
* The explosion stays symmetric under permutations of the axes.
"""
import sys

import numpy as np
import pytest

import inputs
import oracle
from inputs import OUTFLOW, PERIODIC, REFLECT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1808_04960_amd as gw  # noqa: E402
from test_gpu_parity import EPS, flux_bound, rel_l1  # noqa: E402
from parity_bounds import rhs_cell_excess  # noqa: E402


def announce(msg):
    print(f"[gpu-bc] {msg}", file=sys.stderr, flush=True)


BC_GRIDS = {
    1: lambda: inputs.grid1d(200, 0.0, 1.0, [(REFLECT, OUTFLOW)]),
    2: lambda: inputs.grid2d(150, 70, (0.0, 0.0), (1.5, 0.7), [(OUTFLOW, REFLECT), (REFLECT, REFLECT)]),
    3: lambda: inputs.grid3d(66, 45, 30, (0.0, 0.0, 0.0), (1.1, 0.75, 0.5),
                             [(REFLECT, REFLECT), (PERIODIC, PERIODIC), (OUTFLOW, REFLECT)]),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("R", [1, 2, 3])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_rhs_with_boundaries_matches_oracle(ndim, R, prec):
    g = BC_GRIDS[ndim]()
    announce(f"rhs ndim={ndim} R={R} {prec} bc={g.bc[:ndim]}")
    U = inputs.random_smooth(g, seed=200 + 10 * ndim + R)
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


def smallest_grid(ndim, R, h=1.0 / 64):
    """The shortest axes the library accepts for each boundary kind: reflecting
    sides need R + 3 cells, outflow and periodic ones 2."""
    w = R + 3
    if ndim == 1:
        return inputs.grid1d(w, 0.0, w * h, [(REFLECT, REFLECT)])
    if ndim == 2:
        return inputs.grid2d(w, 2, (0.0, 0.0), (w * h, 2 * h), [(REFLECT, OUTFLOW), (OUTFLOW, OUTFLOW)])
    return inputs.grid3d(2, w, 3, (0.0, 0.0, 0.0), (2 * h, w * h, 3 * h),
                         [(OUTFLOW, OUTFLOW), (REFLECT, REFLECT), (PERIODIC, PERIODIC)])


@pytest.mark.parametrize("R", [1, 2, 3])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_smallest_accepted_axes_with_walls_and_outflow(ndim, R):
    """Reflecting axes of exactly R + 3 cells and outflow axes of 2: every ghost
    is a mirror or copy of a cell that is itself near the other wall, and most
    lanes of a run read clamped positions. Right-hand side in both precisions
    within the rounding bounds, three steps within 1e-12 / 1e-5."""
    g = smallest_grid(ndim, R)
    announce(f"smallest axes ndim={ndim} R={R} n={g.n[:ndim]} bc={g.bc[:ndim]}")
    U = inputs.random_smooth(g, seed=500 + 10 * ndim + R)
    dx = g.dx[0]
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


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("R", [1, 2, 3])
def test_shock_tube_run_matches_oracle(R, prec, tol):
    g, U = inputs.shock_tube_1d(200)
    dx = g.dx[0]
    announce(f"shock tube R={R} {prec}")
    Uo = U.copy()
    to, no = oracle.OracleSolver(g, R, 12 * dx, 3 * dx, cfl=0.4).run(Uo, 0.2)
    s = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, cfl=0.4, U0=U)
    n, t = s.run(0.2)
    assert n == no and t == to
    err = rel_l1(s.get_state(), Uo)
    announce(f"  {n} steps, rel L1 vs oracle {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_explosion_3d_matches_oracle(prec, tol):
    """The paper's 3D explosion (Eq. (3d-exp), outflow, CFL 0.3) on 40^3, 12 steps."""
    g, U = inputs.explosion(3, 40)
    dx = g.dx[0]
    announce(f"explosion 40^3 {prec}")
    Uo = U.copy()
    oracle.OracleSolver(g, 2, 12 * dx, 3 * dx, cfl=0.3).run(Uo, 0.25, max_steps=12)
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, cfl=0.3, U0=U)
    n, _ = s.run(0.25, max_steps=12)
    assert n == 12
    err = rel_l1(s.get_state(), Uo)
    announce(f"  rel L1 vs oracle {err:.3e}")
    assert err < tol


def test_explosion_is_symmetric_under_axis_permutations():
    g, U = inputs.explosion(3, 48)
    dx = g.dx[0]
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp64", cfl=0.3, U0=U)
    s.run(0.25, max_steps=40)
    V = s.get_state()
    rho = V[0]
    scale = np.abs(rho).max()
    # (z, y, x) array axes: transposes swap coordinate axes; flips mirror them
    for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)]:
        assert np.abs(rho - rho.transpose(perm)).max() < 1e-12 * scale, perm
    for ax in range(3):
        assert np.abs(rho - np.flip(rho, ax)).max() < 1e-12 * scale, ax


def test_reflecting_wall_is_the_mirror_image():
    n = 96
    g = inputs.grid2d(n, 40, (0.0, 0.0), (1.0, 0.4), [(REFLECT, REFLECT), (PERIODIC, PERIODIC)])
    U = inputs.random_smooth(g, seed=9)
    g2 = inputs.grid2d(2 * n, 40, (-1.0, 0.0), (1.0, 0.4))
    left = U[:, :, ::-1].copy()
    left[1] *= -1.0
    U2 = np.ascontiguousarray(np.concatenate([left, U], axis=2))
    dx = g.dx[0]
    a = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp64", fixed_dt=2e-4, U0=U)
    b = gw.Solver(g2, 2, 12 * dx, 3 * dx, precision="fp64", fixed_dt=2e-4, U0=U2)
    a.run(1.0, max_steps=30)
    b.run(1.0, max_steps=30)
    A, B = a.get_state(), b.get_state()
    assert np.abs(B[:, :, n:] - A).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reflecting_box_conserves_mass_and_energy(prec):
    g = inputs.grid2d(130, 90, (0.0, 0.0), (1.3, 0.9), REFLECT)
    U = inputs.random_smooth(g, seed=21)
    dx = g.dx[0]
    s = gw.Solver(g, 3, 12 * dx, 3 * dx, precision=prec, U0=U)
    m0 = s.conserved_sums()
    s.run(10.0, max_steps=50)
    m1 = s.conserved_sums()
    assert abs(m1[0] - m0[0]) < 1e-13 * abs(m0[0])
    assert abs(m1[3] - m0[3]) < 1e-13 * abs(m0[3])


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_outflow_keeps_a_uniform_flow_bitwise(ndim):
    g = {1: lambda: inputs.grid1d(130, bc=OUTFLOW), 2: lambda: inputs.grid2d(70, 66, bc=OUTFLOW),
         3: lambda: inputs.grid3d(40, 36, 30, bc=OUTFLOW)}[ndim]()
    U = inputs.uniform_state(g)
    s = gw.Solver(g, 2, 0.3, 0.1, precision="fp64", U0=U)
    s.run(1.0, max_steps=10)
    assert np.array_equal(s.get_state(), U)


def test_batch_mixing_boundaries_is_bitwise_the_single_problem_path():
    stream = torch.cuda.Stream()
    probs = [inputs.explosion(2, 64), inputs.isentropic_vortex_2d(64), inputs.explosion(2, 96)]
    solvers = []
    for g, U in probs:
        dx = g.dx[0]
        s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp32", U0=U, stream=stream)
        s.set_end(1e30, 20)
        solvers.append(s)
    b = gw.Batch(stream)
    b.set(solvers)
    b.run(22)
    _, _, ns, err = b.status()
    assert list(ns) == [20, 20, 20] and not err.any()
    for s, (g, U) in zip(solvers, probs):
        dx = g.dx[0]
        ref = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp32", U0=U)
        ref.run(1e30, max_steps=20)
        assert np.array_equal(s.get_state(), ref.get_state())
    b.close()


@pytest.mark.parametrize("R", [2, 3])
def test_explosion_at_the_papers_resolution_follows_the_radial_reference(R):
    """The paper's 3D explosion on 128^3 (CFL 0.3, ell = 12 dx, sigma = 3 dx, to
    t = 0.25), compared as in its Fig. (explosion) with a 1D spherically
    symmetric solution on a fine grid: density along the x axis and the
    diagonal within 1.2 % and 0.9 % (mean absolute difference; shocks smeared
    over a few cells account for most of it), the error halving from 64^3,
    and overshoots along the axes below 2 %."""
    import radial_reference as RR
    from test_reference_solutions import IN, OUT, profiles
    r_ref, rho_ref, _, _, _ = RR.solve(3, IN, OUT, 0.5, 0.25, n=2048)
    errs = {}
    for n in (64, 128):
        g, U = inputs.explosion(3, n)
        dx = g.dx[0]
        s = gw.Solver(g, R, 12 * dx, 3 * dx, precision="fp64", cfl=0.3, U0=U)
        _, t = s.run(0.25)
        assert t == 0.25
        rho = s.get_state()[0]
        (ax, r_ax), (dg, r_dg) = profiles(g, rho)
        errs[n] = (float(np.mean(np.abs(ax - np.interp(r_ax, r_ref, rho_ref))[r_ax < 0.95])),
                   float(np.mean(np.abs(dg - np.interp(r_dg, r_ref, rho_ref))[r_dg < 1.0])))
        announce(f"explosion R={R} n={n}: axis {errs[n][0]:.4f} diagonal {errs[n][1]:.4f} max {rho.max():.4f}")
        if n == 128:
            assert rho.max() < 1.02 and rho.min() > 0.12
        s.close()
    assert errs[128][0] < 0.012 and errs[128][1] < 0.009
    assert errs[128][0] < 0.65 * errs[64][0] and errs[128][1] < 0.65 * errs[64][1]
