"""GPU tests of the C-ABI entry points around the step: the tables a live
context reports, the time step a blocking step returns, runs of any step count
composed from graph replays, resuming from a saved state, the non-physical-state
test hook (alone and inside a batch), batches of problems with non-square
cells, the three-term flux correction against the oracle, and runs on the
default stream.

Parity bars as in test_gpu_parity: 1e-12 (float64) and 1e-5 (float32) relative
L1 for states, 16 eps times the flux scale for one right-hand side.
"""
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


def announce(msg):
    print(f"[gpu-api] {msg}", file=sys.stderr, flush=True)


def rel_l1(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


EPS = {"fp64": 2.0**-53, "fp32": 2.0**-24}


def flux_bound(g, U, gamma=1.4):
    rho, vel, p = inputs.cons_to_prim(g, U, gamma)
    E = U[g.nv - 1]
    total = 0.0
    for d in range(g.ndim):
        un = vel[d]
        F = np.abs(rho * un) + np.abs(un * (E + p)) + sum(np.abs(U[1 + e] * un) for e in range(g.ndim)) + np.abs(p)
        total += F.sum() / g.dx[d]
    return float(total)


# ---------------------------------------------------------------------------
# gpweno_get_tables, gpweno_table_residual
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme,R", [("gp-weno", 1), ("gp-weno", 2), ("gp-weno", 3), ("weno-gp", 2),
                                      ("weno-js", 2), ("gp-ao", 3)])
def test_context_tables_are_those_of_its_axes(scheme, R):
    """Non-square cells: each axis gets the tables of its own ell/dx and
    sigma/dx, equal to the host-only builder's for those ratios."""
    announce(f"get_tables {scheme} R={R}")
    g = inputs.grid2d(40, 30, (0.0, 0.0), (1.0, 1.5))   # dx = 1/40, dy = 1/20
    ell, sig = 0.3, 0.1
    s = gw.Solver(g, R, ell, sig, scheme=scheme, U0=inputs.uniform_state(g))
    for d in range(2):
        t = s.tables(d)
        Rs = 2 if scheme == "gp-ao" else R
        ref = gw.compute_tables(Rs, ell / g.dx[d], sig / g.dx[d], scheme="gp-weno" if scheme == "gp-ao" else scheme)
        n = Rs + 1
        assert np.array_equal(t["w"][0], ref["w+"][:n, :n]) and np.array_equal(t["w"][1], ref["w-"][:n, :n])
        if scheme != "gp-ao":
            assert np.array_equal(t["gamma"][0], ref["gamma+"][:n])
            assert np.array_equal(t["gamma"][1], ref["gamma-"][:n])
        else:
            np.testing.assert_allclose(t["gamma"][0], [0.5 * 0.15 * 0.15, 0.15 * 0.85, 0.5 * 0.15 * 0.15])
        if scheme == "weno-js":
            assert t["P"] is None
        else:
            assert np.array_equal(t["P"], ref["P"][0, :n, :n])
    assert s.table_residual() < 1e-13


def test_badly_conditioned_tables_run_in_float32_only():
    """R = 3 at ell = 80 dx: the binary128 tables hold only about 1e-12 (the
    mirror residual), too little for float64 parity; the context starts in
    float32 and refuses float64."""
    announce("table residual gate")
    g = inputs.grid1d(64)
    dx = g.dx[0]
    s = gw.Solver(g, 3, 80 * dx, 3 * dx, precision="fp32", U0=inputs.uniform_state(g))
    assert s.table_residual() > 1e-13
    with pytest.raises(gw.GpwenoError) as e:
        s.set_options("fp64")
    assert e.value.code == gw.EINVAL
    ok = gw.Solver(g, 3, 40 * dx, 3 * dx, precision="fp64", U0=inputs.uniform_state(g))
    assert ok.table_residual() < 1e-15


# ---------------------------------------------------------------------------
# gpweno_step with dt_out; gpweno_run composed of graph replays
# ---------------------------------------------------------------------------
def test_blocking_step_returns_the_cfl_time_step():
    announce("step dt_out")
    g, U = inputs.isentropic_vortex_2d(64)
    dx = g.dx[0]
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, U0=U)
    o = oracle.OracleSolver(g, 2, 12 * dx, 3 * dx)
    dt = s.step(10.0, wait=True)
    assert dt == pytest.approx(o.dt(U, 0.0, 10.0), rel=1e-14)
    t, dt_rec, n = s.time()
    assert n == 1 and t == dt and dt_rec == dt
    # a step that cannot run (t >= t_final) reports 0 and leaves the state alone
    before = s.get_state()
    assert s.step(t, wait=True) == 0.0
    assert np.array_equal(s.get_state(), before)
    # the last step is clipped to land on t_final
    dt2 = s.step(t + 0.25 * dt, wait=True)
    assert dt2 == pytest.approx(0.25 * dt, rel=1e-12)


@pytest.mark.parametrize("k", [1, 3, 4, 5, 8, 13, 20, 37, 45])
def test_run_takes_exactly_the_steps_asked_for(k):
    """Graph replays of 32, 8, 4 and 1 steps compose any step count; the state
    is bitwise that of k eager steps."""
    announce(f"run max_steps={k}")
    g, U = inputs.isentropic_vortex_2d(48)
    dx = g.dx[0]
    a = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp32", U0=U)
    b = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp32", U0=U)
    n, _ = a.run(1e9, max_steps=k)
    assert n == k
    for _ in range(k):
        b.step(1e9)
    b.synchronize()
    assert a.time() == b.time()
    assert np.array_equal(a.get_state(), b.get_state())


def test_run_to_t_final_lands_exactly():
    announce("run to t_final")
    g, U = inputs.sine_wave_1d(128)
    dx = g.dx[0]
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, U0=U)
    o = oracle.OracleSolver(g, 2, 12 * dx, 3 * dx)
    Uo = U.copy()
    t_o, n_o = o.run(Uo, 0.3)
    n, t = s.run(0.3)
    assert (n, t) == (n_o, t_o)
    assert rel_l1(s.get_state(), Uo) < 1e-12


# ---------------------------------------------------------------------------
# Checkpoint and resume
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_resume_from_a_saved_state_is_bitwise_the_uninterrupted_run(prec):
    """Run k steps, copy the state and time out, bind them in a new context with
    gpweno_set_time, continue: the CFL speed of the restored state is computed
    by the same per-cell function as the stage that produced it, so every
    following dt, and the final state, are bitwise those of the uninterrupted
    run."""
    announce(f"checkpoint/resume {prec}")
    g, U = inputs.isentropic_vortex_2d(64)
    dx = g.dx[0]
    whole = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U)
    whole.run(10.0, max_steps=30)
    first = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U)
    first.run(10.0, max_steps=11)
    t, _, n = first.time()
    saved = first.get_state()
    first.close()
    resumed = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec)
    resumed.set_state(saved, t=t, nsteps=n)
    resumed.run(10.0, max_steps=19)
    assert resumed.time()[0] == whole.time()[0] and resumed.time()[2] == 30
    assert np.array_equal(resumed.get_state(), whole.get_state())


# ---------------------------------------------------------------------------
# gpweno_debug_poison: a non-physical state through the normal error path
# ---------------------------------------------------------------------------
def _near(g, cell, bad, reach):
    """bad lies within `reach` cells of cell along every axis (periodic)."""
    def coords(c):
        out = []
        for d in range(g.ndim):
            out.append(c % g.n[d])
            c //= g.n[d]
        return out
    a, b = coords(cell), coords(bad)
    return all(min(abs(a[d] - b[d]), g.n[d] - abs(a[d] - b[d])) <= reach for d in range(g.ndim))


def test_poisoned_cell_reports_enonphys_with_its_cell():
    announce("poison single")
    g, U = inputs.isentropic_vortex_2d(64)
    dx = g.dx[0]
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, U0=U)
    s.run(10.0, max_steps=3)
    cell = 37 * 64 + 21
    s.debug_poison(cell)
    with pytest.raises(gw.NonPhysicalState):
        s.run(10.0, max_steps=4)
    failed, bad = s.failure()
    assert failed and _near(g, cell, bad, 2 + 3)
    # the condition stays until the state is reset
    with pytest.raises(gw.NonPhysicalState):
        s.time()
    # set_time clears the condition after the caller restores a valid state
    s.set_state(U)
    n, _ = s.run(10.0, max_steps=2)
    assert n == 2 and s.failure() == (False, -1)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_poisoned_problem_fails_alone_in_a_batch(prec):
    """One problem of a batch is poisoned mid-run: it stops with its error flag
    and a flagged cell next to the poisoned one, and every other problem's
    result is bitwise its solo result."""
    announce(f"poison in batch {prec}")
    stream = torch.cuda.Stream()
    probs = [inputs.isentropic_vortex_2d(n) for n in (48, 64, 80)]
    probs.append(inputs.sine_wave_1d(200))
    solvers = []
    for g, U in probs:
        dx = g.dx[0]
        s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U, stream=stream)
        s.set_end(1e30, 12)
        solvers.append(s)
    b = gw.Batch(stream)
    b.set(solvers)
    b.run(4)
    victim = 1
    cell = 40 * 64 + 9
    solvers[victim].debug_poison(cell)
    b.run(10)
    _, _, ns, err = b.status()
    assert err[victim] == 1 and ns[victim] < 12
    assert all(err[i] == 0 and ns[i] == 12 for i in range(len(probs)) if i != victim)
    failed, bad = solvers[victim].failure()
    assert failed and _near(probs[victim][0], cell, bad, 2 + 3)
    for i, (g, U) in enumerate(probs):
        if i == victim:
            continue
        dx = g.dx[0]
        ref = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U)
        ref.run(1e30, max_steps=12)
        assert np.array_equal(solvers[i].get_state(), ref.get_state()), i
    b.close()


# ---------------------------------------------------------------------------
# Batches of problems with non-square cells
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_with_non_square_cells_is_bitwise_the_single_problem_path(prec):
    """Each batched launch covers one direction and takes that direction's
    tables, so problems whose axes have different tables batch like the rest."""
    announce(f"non-square batch {prec}")
    stream = torch.cuda.Stream()
    probs = []
    for i, (nx, ny, ly) in enumerate([(64, 32, 1.0), (64, 32, 1.0), (70, 50, 2.0), (48, 48, 1.0)]):
        g = inputs.grid2d(nx, ny, (0.0, 0.0), (1.0, ly))
        probs.append((g, inputs.random_smooth(g, seed=500 + i)))
    solvers = []
    for g, U in probs:
        s = gw.Solver(g, 2, 0.3, 0.05, precision=prec, U0=U, stream=stream)
        s.set_end(1e30, 9)
        solvers.append(s)
    b = gw.Batch(stream)
    b.set(solvers)
    b.run(9)
    _, _, ns, err = b.status()
    assert list(ns) == [9] * len(probs) and not err.any()
    for s, (g, U) in zip(solvers, probs):
        ref = gw.Solver(g, 2, 0.3, 0.05, precision=prec, U0=U)
        ref.run(1e30, max_steps=9)
        assert np.array_equal(s.get_state(), ref.get_state()), g.n
    b.close()


# ---------------------------------------------------------------------------
# Three-term flux correction (gpweno_options.flux_corr_terms = 3)
# ---------------------------------------------------------------------------
GRIDS = {
    1: lambda: inputs.grid1d(200),
    2: lambda: inputs.grid2d(150, 70, (0.0, 0.0), (1.5, 0.7)),
    3: lambda: inputs.grid3d(66, 45, 30, (0.0, 0.0, 0.0), (1.1, 0.75, 0.5)),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("R", [1, 2, 3])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_three_term_rhs_matches_oracle(ndim, R, prec):
    """56-cell runs (lanes 4..59) with ragged last runs on every axis."""
    g = GRIDS[ndim]()
    announce(f"c6 rhs ndim={ndim} R={R} {prec}")
    U = inputs.random_smooth(g, seed=70 + 10 * ndim + R)
    dx = g.dx[0]
    ref = oracle.OracleSolver(g, R, 12 * dx, 3 * dx, flux_corr_terms=3).rhs(U)
    s = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, U0=U, flux_corr_terms=3)
    got = s.rhs(U)
    err = float(np.abs(got - ref).sum())
    bound = 16 * EPS[prec] * flux_bound(g, U)
    cell = rhs_cell_excess(g, U, got, ref, prec, R, nc=3)
    announce(f"  abs L1 {err:.3e}  bound {bound:.3e}  worst cell {cell:.2f}")
    assert err < bound
    assert cell <= 1.0
    # and it is not the two-term result (on smooth data the two differ by far
    # less than float32 rounding, so only float64 can tell them apart)
    if prec == "fp64":
        two = oracle.OracleSolver(g, R, 12 * dx, 3 * dx).rhs(U)
        assert float(np.abs(two - ref).sum()) > 4 * bound


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_three_term_vortex_steps_match_oracle(prec, tol):
    announce(f"c6 vortex {prec}")
    g, U = inputs.isentropic_vortex_2d(96)
    dx = g.dx[0]
    Uo = U.copy()
    oracle.OracleSolver(g, 3, 12 * dx, 3 * dx, flux_corr_terms=3).run(Uo, 10.0, max_steps=25)
    s = gw.Solver(g, 3, 12 * dx, 3 * dx, precision=prec, U0=U, flux_corr_terms=3)
    n, t = s.run(10.0, max_steps=25)
    assert n == 25
    Ug = s.get_state()
    assert rel_l1(Ug, Uo) < tol
    assert state_cell_excess(g, U, Ug, Uo, prec, t, n) <= 1.0


def test_three_term_reflecting_box_matches_oracle():
    """Reflecting walls need R + 4 mirror ghosts with three terms."""
    announce("c6 reflecting")
    g = inputs.grid2d(40, 36, bc=((inputs.REFLECT, inputs.REFLECT), (inputs.REFLECT, inputs.OUTFLOW)))
    U = inputs.random_smooth(g, seed=91)
    dx = g.dx[0]
    Uo = U.copy()
    oracle.OracleSolver(g, 2, 12 * dx, 3 * dx, flux_corr_terms=3).run(Uo, 1.0, max_steps=8)
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, U0=U, flux_corr_terms=3)
    n, t = s.run(1.0, max_steps=8)
    Ug = s.get_state()
    assert rel_l1(Ug, Uo) < 1e-12
    assert state_cell_excess(g, U, Ug, Uo, "fp64", t, n) <= 1.0


def test_three_term_option_is_validated():
    g = inputs.grid1d(64)
    dx = g.dx[0]
    U = inputs.uniform_state(g)
    for kw in (dict(scheme="weno-js"), dict(scheme="gp-ao", R=3), dict(nonzero_mean=True)):
        R = kw.pop("R", 2)
        with pytest.raises(gw.GpwenoError) as e:
            gw.Solver(g, R, 12 * dx, 3 * dx, U0=U, flux_corr_terms=3, **kw)
        assert e.value.code == gw.EINVAL
    with pytest.raises(gw.GpwenoError):
        gw.Solver(g, 2, 12 * dx, 3 * dx, U0=U, flux_corr_terms=4)
    gr = inputs.grid1d(5, bc=((inputs.REFLECT, inputs.REFLECT),))
    with pytest.raises(gw.GpwenoError):   # R + 4 = 6 mirror ghosts on 5 cells
        gw.Solver(gr, 2, 12 * gr.dx[0], 3 * gr.dx[0], U0=inputs.uniform_state(gr), flux_corr_terms=3)


def test_three_term_batch_is_bitwise_single():
    announce("c6 batch")
    stream = torch.cuda.Stream()
    probs = [inputs.isentropic_vortex_2d(n) for n in (56, 57, 112)]
    solvers = []
    for g, U in probs:
        dx = g.dx[0]
        s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp32", U0=U, stream=stream, flux_corr_terms=3)
        s.set_end(1e30, 7)
        solvers.append(s)
    # a two-term problem in the same batch forms its own group
    g2, U2 = inputs.isentropic_vortex_2d(64)
    s2 = gw.Solver(g2, 2, 12 * g2.dx[0], 3 * g2.dx[0], precision="fp32", U0=U2, stream=stream)
    s2.set_end(1e30, 7)
    b = gw.Batch(stream)
    b.set(solvers + [s2])
    b.run(7)
    _, _, ns, err = b.status()
    assert list(ns) == [7] * 4 and not err.any()
    for s, (g, U) in zip(solvers, probs):
        dx = g.dx[0]
        ref = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp32", U0=U, flux_corr_terms=3)
        ref.run(1e30, max_steps=7)
        assert np.array_equal(s.get_state(), ref.get_state())
    ref2 = gw.Solver(g2, 2, 12 * g2.dx[0], 3 * g2.dx[0], precision="fp32", U0=U2)
    ref2.run(1e30, max_steps=7)
    assert np.array_equal(s2.get_state(), ref2.get_state())
    b.close()


# ---------------------------------------------------------------------------
# The default stream, whose handle is NULL
# ---------------------------------------------------------------------------
def test_default_stream_runs_are_bitwise_the_own_stream_runs():
    """A solver, and a batch of two kinds (so the per-kind streams are used),
    run on the default stream, then move to another stream (new options for
    the solver, a set on the new stream for the batch) and run on; a second
    batch is destroyed right after enqueueing on the default stream. Every
    result is bitwise the same problem's run on a stream of its own."""
    announce("default stream")
    dflt = torch.cuda.default_stream()
    other = torch.cuda.Stream()
    assert dflt.cuda_stream == 0

    def ref_state(g, U, prec, n):
        dx = g.dx[0]
        r = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U)
        r.run(1e30, max_steps=n)
        out = r.get_state()
        r.close()
        return out

    (g, U) = inputs.isentropic_vortex_2d(48)
    dx = g.dx[0]
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp32", U0=U, stream=dflt)
    assert s.run(1e30, max_steps=5)[0] == 5
    s.stream = other
    s.set_options("fp32")
    assert s.run(1e30, max_steps=4)[0] == 4
    assert np.array_equal(s.get_state(), ref_state(g, U, "fp32", 9))
    s.close()

    probs = [(inputs.isentropic_vortex_2d(48), "fp32"), (inputs.isentropic_vortex_2d(64), "fp64"),
             (inputs.isentropic_vortex_2d(40), "fp32")]
    solvers = []
    for (g, U), prec in probs:
        dx = g.dx[0]
        sv = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U, stream=dflt)
        sv.set_end(1e30, 10)
        solvers.append(sv)
    b = gw.Batch(dflt)
    b.set(solvers)
    b.run(3)
    b.stream = other
    for sv, (_, prec) in zip(solvers, probs):
        sv.stream = other
        sv.set_options(prec)
    b.set(solvers)
    b.run(7)
    _, _, ns, err = b.status()
    assert list(ns) == [10] * 3 and not err.any()
    for sv, ((g, U), prec) in zip(solvers, probs):
        assert np.array_equal(sv.get_state(), ref_state(g, U, prec, 10))
    b.close()

    (g, U), prec = probs[1]
    dx = g.dx[0]
    sv = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U, stream=dflt)
    sv.set_end(1e30, 6)
    b2 = gw.Batch(dflt)
    b2.set([sv])
    b2.run(6)
    b2.close()
    assert np.array_equal(sv.get_state(), ref_state(g, U, prec, 6))
    for x in solvers + [sv]:
        x.close()
