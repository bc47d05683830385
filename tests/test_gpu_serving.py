"""Batched execution and the continuous-batching server on the GPU.

* A batch of problems of mixed size, R and initial data gives, for each problem,
  bitwise the state the single-problem path gives: every block of the batched
  kernel runs the single-problem sweep on its own problem's data.
* Through the server, a request's result is bitwise the same alone and in a mix
  of other requests arriving while it runs.
* Batched results agree with the CPU oracle (1e-12 fp64, 1e-5 fp32).
* The batch's limits (64 kinds, 4096 problems) hold, and larger sets are
  refused; an empty batch runs nothing.
"""
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
from paper_1808_04960_amd.serve import GpuExecutor, Server  # noqa: E402


def announce(msg):
    print(f"[gpu-serving] {msg}", file=sys.stderr, flush=True)


def make_req(rid, n, R, steps, kind, arrival=0.0, seed=None):
    if kind == "vortex":
        g = inputs.grid2d(n, n, (-5.0, -5.0), (5.0, 5.0))
    else:
        g = inputs.grid2d(n, n)
    return inputs.Request(rid, arrival, n, R, steps, kind, g, seed if seed is not None else 1000 + rid)


MIX = [(64, 1, 23, "vortex"), (96, 2, 31, "quadrant"), (128, 3, 17, "vortex"), (80, 2, 40, "quadrant"),
       (64, 3, 29, "quadrant"), (112, 1, 35, "vortex"), (128, 2, 26, "vortex"), (72, 3, 33, "vortex")]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_is_bitwise_the_single_problem_path(prec):
    announce(f"batch vs single, {prec}")
    stream = torch.cuda.Stream()
    reqs = [make_req(i, *m) for i, m in enumerate(MIX)]
    solvers = []
    for r in reqs:
        dx = r.grid.dx[0]
        s = gw.Solver(r.grid, r.R, 12 * dx, 3 * dx, precision=prec, positivity_fallback=(r.kind == "quadrant"),
                      U0=r.state(), stream=stream)
        s.set_end(1e30, r.steps)
        solvers.append(s)
    b = gw.Batch(stream)
    b.set(solvers)
    b.run(max(r.steps for r in reqs) + 3)   # extra steps must be no-ops for finished problems
    t, dt, ns, err = b.status()
    assert list(ns) == [r.steps for r in reqs] and not err.any()
    for r, s, ti in zip(reqs, solvers, t):
        dx = r.grid.dx[0]
        ref = gw.Solver(r.grid, r.R, 12 * dx, 3 * dx, precision=prec, positivity_fallback=(r.kind == "quadrant"),
                        U0=r.state())
        n, tr = ref.run(1e30, max_steps=r.steps)
        assert n == r.steps and tr == ti
        assert np.array_equal(s.get_state(), ref.get_state()), r
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_3d_is_bitwise_the_single_problem_path(prec):
    """3D problems through the batched kernels: every y/z block (8 x columns in
    float32, 4 in float64) and every ragged pencil group and run segment of a
    problem must be owned by that problem and reproduce its single-problem
    result bitwise; periodic and outflow problems form separate kernel groups."""
    announce(f"3D batch vs single, {prec}")
    stream = torch.cuda.Stream()
    probs = []
    for i, (nx, ny, nz) in enumerate([(41, 20, 18), (33, 33, 24), (20, 45, 30), (67, 12, 9)]):
        g = inputs.grid3d(nx, ny, nz, (0.0, 0.0, 0.0), (nx / 32, ny / 32, nz / 32))  # square cells, exactly
        probs.append((g, inputs.random_smooth(g, seed=300 + i)))
    probs.append(inputs.explosion(3, 26))
    solvers = []
    for g, U in probs:
        dx = g.dx[0]
        s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U, stream=stream)
        s.set_end(1e30, 6)
        solvers.append(s)
    b = gw.Batch(stream)
    b.set(solvers)
    b.run(7)
    _, _, ns, err = b.status()
    assert list(ns) == [6] * len(probs) and not err.any()
    for s, (g, U) in zip(solvers, probs):
        dx = g.dx[0]
        ref = gw.Solver(g, 2, 12 * dx, 3 * dx, precision=prec, U0=U)
        ref.run(1e30, max_steps=6)
        assert np.array_equal(s.get_state(), ref.get_state()), g.n
    b.close()


def test_server_alone_equals_mix_bitwise():
    announce("server alone vs mix")
    # arrivals closer together than a job lasts: later requests join while earlier
    # ones run, and wait for slots when all 5 are taken
    reqs = [make_req(i, *m, arrival=0.0002 * i) for i, m in enumerate(MIX)]
    budget = 1 << 30
    mix = Server(GpuExecutor("fp32"), hbm_budget=budget, max_slots=5, steps_per_tick=4).run(reqs, keep_results=True)
    assert all(j.status == "done" for j in mix.jobs)
    assert mix.peak_active >= 3      # requests really overlapped on the device
    for j in mix.jobs:
        alone = Server(GpuExecutor("fp32"), hbm_budget=budget, max_slots=5, steps_per_tick=7).run(
            [make_req(j.req.rid, *MIX[j.req.rid], arrival=0.0)], keep_results=True)
        assert np.array_equal(alone.jobs[0].result, j.result), j.req.rid


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_batched_results_match_oracle(prec, tol):
    announce(f"batched vs oracle, {prec}")
    reqs = [make_req(0, 96, 2, 30, "vortex"), make_req(1, 64, 3, 25, "quadrant"), make_req(2, 80, 1, 40, "vortex")]
    rep = Server(GpuExecutor(prec), hbm_budget=1 << 30, max_slots=8, steps_per_tick=8).run(reqs, keep_results=True)
    for j in rep.jobs:
        r = j.req
        dx = r.grid.dx[0]
        U = r.state()
        oracle.OracleSolver(r.grid, r.R, 12 * dx, 3 * dx, positivity_fallback=(r.kind == "quadrant")).run(
            U, 1e30, max_steps=r.steps)
        err = np.abs(j.result - U).sum() / np.abs(U).sum()
        assert err < tol, (r.rid, err)


def test_poisson_stream_small():
    announce("small Poisson stream")
    reqs = inputs.serving_stream(count=40, rate=200.0, seed=5, sizes=(64, 128, 256), steps=(20, 60))
    rep = Server(GpuExecutor("fp32"), hbm_budget=256 << 20, max_slots=16, steps_per_tick=8).run(reqs)
    s = rep.summary()
    assert s["completed"] == 40 and s["failed"] == 0
    assert rep.peak_bytes <= 256 << 20
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_set_changes_reuse_the_captured_step_graph():
    """Problems join and leave between batched runs: the set is rewritten into
    the batch's device work tables by stream-ordered copies, the captured step
    graph keeps serving it (one capture for one kind of problem), and every
    problem's result is bitwise its solo result. A new kind (R = 3) adds one
    capture, and set changes within those two kinds again keep the graph."""
    announce("set changes without recapture")
    stream = torch.cuda.Stream()

    def mk(n, limit, R=2):
        g, U = inputs.isentropic_vortex_2d(n)
        dx = g.dx[0]
        s = gw.Solver(g, R, 12 * dx, 3 * dx, precision="fp32", U0=U, stream=stream)
        s.set_end(1e30, limit)
        return s, (g, U, R, limit)

    a0, ia0 = mk(64, 5)
    a1, ia1 = mk(80, 15)
    a2, ia2 = mk(96, 10)
    b = gw.Batch(stream)
    b.set([a0, a1, a2])
    b.run(5)
    c0, ic0 = mk(72, 10)
    b.set([a1, a2, c0])          # a0 finished and left, c0 joined
    b.run(5)
    b.set([a1, c0])              # a2 finished and left
    b.run(5)
    assert b.captures() == 1
    d3, id3 = mk(64, 4, R=3)     # a new kind of problem
    b.set([a1, c0, d3])
    b.run(4)
    assert b.captures() == 2
    _, _, ns, err = b.status()
    assert list(ns) == [15, 10, 4] and not err.any()
    e3, ie3 = mk(56, 6, R=3)
    f2, if2 = mk(88, 3)
    b.set([c0, e3, f2, a1])      # d3 finished and left, e3 and f2 joined
    b.run(6)
    assert b.captures() == 2
    _, _, ns, err = b.status()
    assert list(ns) == [10, 6, 3, 15] and not err.any()
    for s, (g, U, R, limit) in ((a0, ia0), (a1, ia1), (a2, ia2), (c0, ic0), (d3, id3), (e3, ie3), (f2, if2)):
        ref = gw.Solver(g, R, 12 * g.dx[0], 3 * g.dx[0], precision="fp32", U0=U)
        ref.run(1e30, max_steps=limit)
        assert s.time()[2] == limit
        assert np.array_equal(s.get_state(), ref.get_state()), (g.n, R)
    b.close()


def test_new_kinds_join_while_the_step_graph_runs():
    """Kinds join a batch whose step graph was launched and not waited for, so
    each new kind replaces a graph that may still be running: the old graph
    must finish first, and every problem's result is bitwise its solo result."""
    announce("new kinds while the step graph runs")
    stream = torch.cuda.Stream()

    def mk(n, limit, R, prec="fp32"):
        g, U = inputs.isentropic_vortex_2d(n)
        dx = g.dx[0]
        s = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, U0=U, stream=stream)
        s.set_end(1e30, limit)
        return s, (g, U, R, limit, prec)

    probs = [mk(64, 30, 1), mk(72, 30, 2)]
    b = gw.Batch(stream)
    b.set([p for p, _ in probs])
    b.run(10)
    for extra, k in ((mk(56, 20, 3), 10), (mk(64, 12, 2, "fp64"), 10), (mk(48, 9, 1, "fp64"), 12)):
        probs.append(extra)
        b.set([p for p, _ in probs])
        b.run(k)
    assert b.captures() == 4
    _, _, ns, err = b.status()
    assert list(ns) == [30, 30, 20, 12, 9] and not err.any()
    for s, (g, U, R, limit, prec) in probs:
        ref = gw.Solver(g, R, 12 * g.dx[0], 3 * g.dx[0], precision=prec, U0=U)
        ref.run(1e30, max_steps=limit)
        assert np.array_equal(s.get_state(), ref.get_state()), (g.n, R, prec)
    b.close()


def test_batch_mixing_dimensions_precisions_and_sizes_is_bitwise_single():
    """One batch holding 1D, 2D and 3D problems in both precisions, including
    axes of a few cells: each kind is its own group with its own step graph
    (3, 6 and 9 launches per step) on its own stream, and a set change that
    swaps problems for larger or smaller ones of the same kinds only updates the
    launch grids. Every problem is bitwise its solo run."""
    announce("batch mixing dimensions, precisions and sizes")
    stream = torch.cuda.Stream()

    def grid(shape, h=1.0 / 64):
        hi = [n * h for n in shape]
        if len(shape) == 1:
            return inputs.grid1d(shape[0], 0.0, hi[0])
        if len(shape) == 2:
            return inputs.grid2d(shape[0], shape[1], (0.0, 0.0), tuple(hi))
        return inputs.grid3d(*shape, (0.0, 0.0, 0.0), tuple(hi))

    def mk(shape, prec, R, limit, seed):
        g = grid(shape)
        U = inputs.random_smooth(g, seed=seed)
        dx = g.dx[0]
        s = gw.Solver(g, R, 12 * dx, 3 * dx, precision=prec, U0=U, stream=stream)
        s.set_end(1e30, limit)
        return s, (g, U, prec, R, limit)

    first = [mk((300,), "fp64", 2, 9, 1), mk((5,), "fp32", 3, 7, 2), mk((70, 33), "fp32", 2, 8, 3),
             mk((3, 90), "fp64", 2, 6, 4), mk((20, 13, 11), "fp32", 2, 5, 5), mk((9, 2, 30), "fp64", 2, 7, 6)]
    b = gw.Batch(stream)
    b.set([s for s, _ in first])
    b.run(4)
    # same kinds, other sizes: the first three leave, larger and smaller ones join
    second = [mk((1000,), "fp64", 2, 6, 7), mk((2,), "fp32", 3, 5, 8), mk((130, 21), "fp32", 2, 4, 9)]
    keep = first[3:]
    b.set([s for s, _ in keep + second])
    b.run(10)
    assert b.captures() == 1
    _, _, ns, err = b.status()
    assert list(ns) == [info[4] for _, info in keep + second] and not err.any()
    for s, (g, U, prec, R, limit) in first[:3]:
        assert s.time()[2] == 4   # left the batch after four steps
    for s, (g, U, prec, R, limit) in first + second:
        ref = gw.Solver(g, R, 12 * g.dx[0], 3 * g.dx[0], precision=prec, U0=U)
        ref.run(1e30, max_steps=s.time()[2])
        assert np.array_equal(s.get_state(), ref.get_state()), (g.n, prec, R)
    b.close()


def test_batch_limits_64_kinds_and_4096_problems():
    """The batch's limits. 64 kinds of problems (1D, tables differing in ell,
    so each kind has its own graphs and stream) and then 4096 problems of one
    kind run together, each sampled problem bitwise its single-problem result;
    a 65th kind and a 4097th problem are refused (EINVAL), and the batch keeps
    serving the set it had."""
    announce("batch limits: 64 kinds, 4096 problems")
    stream = torch.cuda.Stream()
    g, U = inputs.sine_wave_1d(64)
    _, U2 = inputs.sine_wave_1d(64, amp=0.1)
    dx = g.dx[0]

    def solo(ell, prec, U0, n):
        r = gw.Solver(g, 2, ell, 3 * dx, precision=prec, U0=U0)
        r.run(1e30, max_steps=n)
        out = r.get_state()
        r.close()
        return out

    ells = [(6 + 0.25 * i) * dx for i in range(64)]
    kinds = []
    for ell in ells:
        s = gw.Solver(g, 2, ell, 3 * dx, precision="fp32", U0=U, stream=stream)
        s.set_end(1e30, 9)
        kinds.append(s)
    b = gw.Batch(stream)
    b.set(kinds)
    b.run(9)
    _, _, ns, err = b.status()
    assert list(ns) == [9] * 64 and not err.any()
    extra = gw.Solver(g, 2, 40 * dx, 3 * dx, precision="fp32", U0=U, stream=stream)
    with pytest.raises(gw.GpwenoError) as e:
        b.set(kinds + [extra])
    assert e.value.code == gw.EINVAL
    b.run(2)   # the old set, all at their step limit: nothing moves
    _, _, ns, err = b.status()
    assert list(ns) == [9] * 64 and not err.any()
    for i in (0, 21, 42, 63):
        assert np.array_equal(kinds[i].get_state(), solo(ells[i], "fp32", U, 9)), i
    b.close()
    for s in kinds:
        s.close()

    many = []
    for i in range(4096):
        s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp64", U0=U if i % 2 == 0 else U2, stream=stream)
        s.set_end(1e30, 5)
        many.append(s)
    b = gw.Batch(stream)
    b.set(many)
    b.run(5)
    _, _, ns, err = b.status()
    assert len(ns) == 4096 and (ns == 5).all() and not err.any()
    with pytest.raises(gw.GpwenoError) as e:
        b.set(many + [extra])
    assert e.value.code == gw.EINVAL
    ref = {0: solo(12 * dx, "fp64", U, 5), 1: solo(12 * dx, "fp64", U2, 5)}
    for i in (0, 1, 2047, 2048, 4094, 4095):
        assert np.array_equal(many[i].get_state(), ref[i % 2]), i
    b.close()
    for s in many + [extra]:
        s.close()


def test_empty_batch_runs_nothing():
    """A batch with no problems (never set, set empty, or emptied after its
    graphs were captured) runs nothing and reports nothing; a problem that
    left it keeps the state it had."""
    announce("empty batch")
    stream = torch.cuda.Stream()
    b = gw.Batch(stream)
    b.run(3)
    b.set([])
    b.run(2)
    t, dt, ns, err = b.status()
    assert len(t) == len(dt) == len(ns) == len(err) == 0
    g, U = inputs.isentropic_vortex_2d(40)
    dx = g.dx[0]
    s = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp32", U0=U, stream=stream)
    s.set_end(1e30, 100)
    b.set([s])
    b.run(3)
    b.set([])
    b.run(4)
    assert len(b.status()[2]) == 0
    ref = gw.Solver(g, 2, 12 * dx, 3 * dx, precision="fp32", U0=U)
    ref.run(1e30, max_steps=3)
    assert s.time()[2] == 3
    assert np.array_equal(s.get_state(), ref.get_state())
    b.close()
    s.close()
    ref.close()
