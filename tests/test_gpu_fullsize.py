"""Full-size parity at the benchmark-scale configurations, on sampled outputs.

The GPU runs the whole grid in the launch configuration the benchmark times
(graph-replayed gpweno_run steps, or one right-hand side). The oracle then
recomputes sampled boxes of cells one box at a time. A cell's right-hand side
depends only on cells within G = R+3 along each axis, so a box padded by G
(periodic padding that never reaches the compared interior) gives the oracle
value exactly. One SSP-RK3 step chains three right-hand sides, so there the
padding is 3G and the oracle takes the step with the GPU's dt. The dt itself
is checked against the oracle's CFL rule on the full state.
"""
import sys

import numpy as np
import pytest

import inputs
import oracle
from parity_bounds import EPS as _EPS, conserved_totals_bound, local_flux_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1808_04960_amd as gw  # noqa: E402


def announce(msg):
    print(f"[gpu-fullsize] {msg}", file=sys.stderr, flush=True)


CONFIGS = {
    "C2-vortex-512": (lambda: inputs.isentropic_vortex_2d(512), 2),
    "C3-kh-2048x1024": (lambda: inputs.kelvin_helmholtz_2d(2048, 1024), 3),
    "C4-wave-256": (lambda: inputs.density_wave_3d(256), 2),
    "C4-vortex-256": (lambda: inputs.isentropic_vortex_3d(256), 2),
    # the largest axis the library accepts (2^24 cells): 289,262 runs per pencil
    "max-axis-1d-2^24": (lambda: inputs.sine_wave_1d(1 << 24), 2),
}


def box_indices(grid, starts, size, pad):
    """Per-axis index arrays (slowest axis first, as the state is laid out)."""
    idx = []
    for d in reversed(range(grid.ndim)):
        idx.append(np.arange(starts[d] - pad, starts[d] + size + pad) % grid.n[d])
    return idx


def box_grid(grid, size, pad):
    n = [size + 2 * pad] * grid.ndim
    lo = [0.0] * grid.ndim
    hi = [n[d] * grid.dx[d] for d in range(grid.ndim)]
    if grid.ndim == 1:
        return inputs.grid1d(n[0], 0.0, hi[0])
    if grid.ndim == 2:
        return inputs.grid2d(n[0], n[1], lo, hi)
    return inputs.grid3d(n[0], n[1], n[2], lo, hi)


def extract(U, idx):
    return np.ascontiguousarray(U[(slice(None),) + np.ix_(*idx)])


def interior(A, ndim, pad, size):
    sl = (slice(None),) + tuple(slice(pad, pad + size) for _ in range(ndim))
    return A[sl]


def sample_starts(grid, rng, count):
    """Box corners: one straddling the periodic seam, the rest random."""
    out = [[grid.n[d] - 3 for d in range(grid.ndim)]]
    for _ in range(count - 1):
        out.append([int(rng.integers(0, grid.n[d])) for d in range(grid.ndim)])
    return out


EPS = {"fp64": 2.0**-53, "fp32": 2.0**-24}


def flux_scale(g, U, gamma=1.4):
    rho, vel, p = inputs.cons_to_prim(g, U, gamma)
    E = U[g.nv - 1]
    tot = 0.0
    for d in range(g.ndim):
        un = vel[d]
        F = np.abs(rho * un) + np.abs(un * (E + p)) + sum(np.abs(U[1 + e] * un) for e in range(g.ndim)) + np.abs(p)
        tot += F.sum() / g.dx[d]
    return float(tot)


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fullsize_rhs_sampled(name, prec):
    make, R = CONFIGS[name]
    g, U = make()
    announce(f"{name} {prec}: full-size right-hand side, n={g.n[:g.ndim]}")
    dx = g.dx[0]
    s = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, U0=U)
    L = s.rhs(U)
    G = R + 3
    size = 12 if g.ndim < 3 else 6
    bg = box_grid(g, size, G)
    o = oracle.OracleSolver(bg, R, 12 * dx, 3 * dx)
    rng = np.random.default_rng(1)
    for starts in sample_starts(g, rng, 4):
        idx = box_indices(g, starts, size, G)
        Ub = extract(U, idx)
        ref = interior(o.rhs(Ub), g.ndim, G, size)
        got = interior(extract(L, idx), g.ndim, G, size)
        err = float(np.abs(got - ref).sum())
        bound = 16 * EPS[prec] * flux_scale(bg, interior(Ub, g.ndim, G, size))
        assert err < bound, (starts, err, bound)
        # per cell: 32 eps of the largest face flux within reach (parity_bounds)
        cell_scale = interior(local_flux_scale(bg, Ub, R + 3)[None], g.ndim, G, size)
        assert np.all(np.abs(got - ref) <= 32 * _EPS[prec] * cell_scale), starts


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_fullsize_step_sampled(name, prec, tol):
    make, R = CONFIGS[name]
    g, U = make()
    announce(f"{name} {prec}: one full-size SSP-RK3 step through gpweno_run")
    dx = g.dx[0]
    s = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, U0=U)
    n, t = s.run(1e9, max_steps=1)
    assert n == 1
    t_gpu, dt_gpu, _ = s.time()
    assert t_gpu == dt_gpu
    # the CFL time step of the full state (float64 on both sides)
    dt_ref = oracle.OracleSolver(g, R, 12 * dx, 3 * dx).dt(U, 0.0, 1e9)
    assert abs(dt_gpu - dt_ref) <= 1e-14 * dt_ref
    U1 = s.get_state()
    G = 3 * (R + 3)
    size = 10 if g.ndim < 3 else 4
    bg = box_grid(g, size, G)
    o = oracle.OracleSolver(bg, R, 12 * dx, 3 * dx)
    rng = np.random.default_rng(2)
    num = den = 0.0
    for starts in sample_starts(g, rng, 4):
        idx = box_indices(g, starts, size, G)
        Ub = extract(U, idx)
        o.step(Ub, dt_gpu)
        ref = interior(Ub, g.ndim, G, size)
        got = interior(extract(U1, idx), g.ndim, G, size)
        num += float(np.abs(got - ref).sum())
        den += float(np.abs(ref).sum())
        # per cell: one step moves each cell by dt L, so the right-hand-side
        # bound times dt (the three stages' weights sum to one), plus float64
        # rounding of the stage combinations
        S = float(local_flux_scale(bg, Ub, 3 * (R + 3)).max())
        umax = np.abs(ref).reshape(g.nv, -1).max(axis=1)[(slice(None),) + (None,) * g.ndim]
        assert np.all(np.abs(got - ref) <= 32 * _EPS[prec] * dt_gpu * S + 8 * _EPS["fp64"] * umax), starts
    assert num / den < tol, num / den


# States of more than 2^31 float64 values, tiled from a benchmark-scale state:
# 48 x 48 copies of the 512^2 vortex (24576^2 cells, 4 fields: 2.4e9 values,
# 19.3 GB per array) and 3 x 3 x 3 copies of the 256^3 density wave (768^3
# cells, 5 fields: 2.3e9 values, 18.1 GB per array), so every kernel of a step
# indexes past 2^31 elements. A tiled field is periodic with the tile's period,
# so the CFL time step is the tile's and the conserved totals are the number of
# tiles times the tile's.
BIG = {
    "2d-vortex-24576^2": (lambda: inputs.isentropic_vortex_2d(512), 48, 10),
    "3d-wave-768^3": (lambda: inputs.density_wave_3d(256), 3, 4),
}


def tiled_grid(gt, tiles):
    n = [gt.n[d] * tiles for d in range(gt.ndim)]
    lo = [gt.lo[d] for d in range(gt.ndim)]
    hi = [gt.lo[d] + n[d] * gt.dx[d] for d in range(gt.ndim)]
    if gt.ndim == 2:
        return inputs.grid2d(n[0], n[1], lo, hi)
    return inputs.grid3d(n[0], n[1], n[2], lo, hi)


@pytest.mark.parametrize("name", list(BIG))
def test_state_beyond_2_31_values_step_sampled(name):
    make, tiles, size = BIG[name]
    gt, Ut = make()
    R = 2
    g = tiled_grid(gt, tiles)
    ncell = int(np.prod(g.n[:g.ndim]))
    assert g.nv * ncell > 2**31
    dx = gt.dx[0]
    announce(f"{name} ({g.nv * ncell:.3e} values): tiling on the host")
    U = np.tile(Ut, (1,) + (tiles,) * g.ndim)
    s = gw.Solver(g, R, 12 * dx, 3 * dx, precision="fp64")
    dt_ref = oracle.OracleSolver(gt, R, 12 * dx, 3 * dx).dt(Ut, 0.0, 1e9)
    ntile = tiles ** g.ndim
    tile_totals = Ut.reshape(g.nv, -1).sum(axis=1) * ntile
    scale = np.abs(Ut).reshape(g.nv, -1).sum(axis=1) * ntile
    G = 3 * (R + 3)
    bg = box_grid(g, size, G)
    o = oracle.OracleSolver(bg, R, 12 * dx, 3 * dx)
    # boxes: across the seam at the last cells (the largest indices), inside
    # the last tile along each axis, and two at random
    rng = np.random.default_rng(5)
    n = g.n
    far = [[n[0] - 40] + [n[d] - 20 for d in range(1, g.ndim)],
           [n[0] // 3] + [n[d] - 40 for d in range(1, g.ndim)]]
    starts = sample_starts(g, rng, 3) + far
    try:
        for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
            announce(f"  {prec}: upload, one step through gpweno_run, sampled boxes")
            s.set_options(prec)
            s.set_state(U)
            sums0 = s.conserved_sums()
            np.testing.assert_allclose(sums0, tile_totals, rtol=1e-12, atol=1e-12 * scale.max())
            nst, _ = s.run(1e9, max_steps=1)
            assert nst == 1
            t_gpu, dt_gpu, _ = s.time()
            assert abs(dt_gpu - dt_ref) <= 1e-14 * dt_ref
            sums1 = s.conserved_sums()
            s.synchronize()
            # periodic: one step changes the float64 totals only by the
            # rounding of the per-cell updates and of the sums
            assert np.all(np.abs(sums1 - sums0) <= conserved_totals_bound(ncell, 1, scale)), (sums0, sums1)
            announce(f"    totals changed by {float((np.abs(sums1 - sums0) / scale).max()):.2e} of sum|U_k|")
            num = den = 0.0
            for st in starts:
                idx = box_indices(g, st, size, G)
                Ub = extract(U, idx)
                o.step(Ub, dt_gpu)
                ref = interior(Ub, g.ndim, G, size)
                box = s.state
                for a, ia in enumerate(idx):
                    box = box.index_select(1 + a, torch.as_tensor(ia, device=s.state.device))
                got = interior(box.cpu().numpy(), g.ndim, G, size)
                num += float(np.abs(got - ref).sum())
                den += float(np.abs(ref).sum())
                S = float(local_flux_scale(bg, Ub, G).max())
                umax = np.abs(ref).reshape(g.nv, -1).max(axis=1)[(slice(None),) + (None,) * g.ndim]
                assert np.all(np.abs(got - ref) <= 32 * _EPS[prec] * dt_gpu * S + 8 * _EPS["fp64"] * umax), (prec, st)
            announce(f"    sampled boxes: relative L1 {num / den:.2e}")
            assert num / den < tol, (prec, num / den)
    finally:
        s.close()
        del U
