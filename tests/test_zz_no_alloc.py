"""The entry point that allocates nothing (gpweno_step_noalloc), through the
C ABI: its steps of a caller-passed state, with the stage states and the
direction accumulator in the library's fixed device scratch, give bitwise the
states (and the same times) of gpweno_step on a bound state with a caller
workspace, on two problems in a row, the second smaller, sharing that scratch;
and both agree with the oracle to the float64 parity bar. A grid whose step
scratch exceeds the library's is refused."""
import ctypes
import sys

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1808_04960_amd as gw  # noqa: E402


def announce(msg):
    print(f"[gpu-noalloc] {msg}", file=sys.stderr, flush=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_step_equals_the_workspace_step(prec):
    problems = [
        ("2D 200x150 R3", inputs.grid2d(200, 150, (0.0, 0.0), (1.0, 0.75)), 3, 4),
        ("2D 64x48 R2 (smaller)", inputs.grid2d(64, 48, (0.0, 0.0), (1.0, 0.75)), 2, 5),
    ]
    for name, g, R, nsteps in problems:
        announce(f"{name} {prec}: {nsteps} steps, workspace vs no-alloc")
        U = inputs.random_smooth(g, seed=11 + R)
        dx = g.dx[0]
        a = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, U0=U)
        b = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, U0=U)
        ext = torch.tensor(U, dtype=torch.float64, device=b.device)   # a state b is not bound to
        torch.cuda.synchronize()
        for _ in range(nsteps):
            a.step(1e9)
            b.step_noalloc(1e9, ext)
        a.synchronize()
        b.synchronize()
        Ua = a.get_state()
        Ub = ext.cpu().numpy()
        assert a.time() == b.time()
        assert np.array_equal(Ua, Ub)
        assert np.array_equal(b.get_state(), U)   # its own bound state untouched
        if prec == "fp64":
            Uo = U.copy()
            oracle.OracleSolver(g, R, 12 * dx, 3 * dx).run(Uo, 1e9, max_steps=nsteps)
            assert float(np.abs(Ub - Uo).sum() / np.abs(Uo).sum()) < 1e-12


def test_noalloc_step_refuses_a_grid_beyond_its_scratch():
    g = inputs.grid2d(1024, 1024)   # 3 arrays of 4 x 2^20 doubles: 96 MiB > 64 MiB
    s = gw.Solver(g, 2, 12 * g.dx[0], 3 * g.dx[0], U0=inputs.uniform_state(g))
    with pytest.raises(gw.GpwenoError) as e:
        s.step_noalloc(1.0)
    assert e.value.code == gw.EINVAL and "scratch" in str(e.value)
    assert gw.lib().gpweno_step_noalloc(None, None, 1.0) == gw.EINVAL
    assert gw.lib().gpweno_step_noalloc(s._ctx, ctypes.c_void_p(8 + 4), 1.0) == gw.EINVAL
