"""Right-hand-side parity over seeded random configurations (GPU against the
CPU oracle, per cell): dimension, axis lengths (ragged runs and pencil groups,
axes down to a few cells), cell aspect ratio, boundary kind per side
(periodic, outflow, reflecting), stencil radius, scheme with GP indicators of
zero mean (GP-WENO, WENO-GP, adaptive-order GP), flux-correction terms, GP
length scales and precision, each on smooth random data of moderate or large
amplitude. Every configuration must meet the per-cell bound of parity_bounds
(32 eps of the largest face flux within reach).

GP-AO keeps the normalisation (log-det) constants of its indicators, which are
negative for sigma above about 1.6 dx (the 7-point one: -1.3 at 1.8 dx, -9.6
at 3 dx), so eps + beta vanishes where the data's fit term equals minus that
constant, and the weights 1/(eps + beta)^2 then amplify any rounding of the
data without bound: the oracle's own result moves by as much under relative
perturbations of its data of the sweep's eps. There a cell may also differ by
four times that spread (8 perturbations of every value by eps times a
uniform number in [-1, 1])."""
import sys

import numpy as np
import pytest

import inputs
import oracle
from parity_bounds import EPS, conserved_totals_bound, local_flux_scale, state_cell_excess

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1808_04960_amd as gw  # noqa: E402

NCASES = 36
MAX_N = {1: 150, 2: 70, 3: 24}


def announce(msg):
    print(f"[gpu-random] {msg}", file=sys.stderr, flush=True)


def draw(i):
    rng = np.random.default_rng(7000 + i)
    ndim = int(rng.integers(1, 4))
    scheme = ["gp-weno", "weno-gp", "gp-ao"][int(rng.integers(0, 3))]
    R = int(rng.integers(2, 4)) if scheme == "gp-ao" else int(rng.integers(1, 4))
    nc = 3 if scheme != "gp-ao" and rng.random() < 0.35 else 2
    prec = ["fp64", "fp32"][int(rng.integers(0, 2))]
    n, bc, hi = [], [], []
    h = 1.0 / 64
    for d in range(ndim):
        if rng.random() < 0.5:
            b = (inputs.PERIODIC, inputs.PERIODIC)
            lo_n = 2
        else:
            b = tuple(int(x) for x in rng.choice([inputs.OUTFLOW, inputs.REFLECT], size=2))
            lo_n = R + 1 + nc
        nd = int(rng.integers(lo_n, MAX_N[ndim] + 1))
        n.append(nd)
        bc.append(b)
        hi.append(nd * h * float(rng.uniform(1.0, 1.5)))   # cells up to 1.5 : 1
    if ndim == 1:
        g = inputs.grid1d(n[0], 0.0, hi[0], bc)
    elif ndim == 2:
        g = inputs.grid2d(n[0], n[1], (0.0, 0.0), tuple(hi), bc)
    else:
        g = inputs.grid3d(n[0], n[1], n[2], (0.0, 0.0, 0.0), tuple(hi), bc)
    dxmax = max(g.dx[:ndim])
    ell = float(rng.uniform(6.0, 16.0)) * dxmax
    sigma = float(rng.uniform(2.0, 3.5)) * dxmax
    amp = float(rng.choice([0.1, 0.25]))
    U = inputs.random_smooth(g, seed=9000 + i, amp=amp)
    return dict(g=g, U=U, R=R, scheme=scheme, nc=nc, prec=prec, ell=ell, sigma=sigma, amp=amp)


@pytest.mark.parametrize("i", range(NCASES))
def test_random_configuration_rhs_matches_oracle(i):
    c = draw(i)
    g = c["g"]
    announce(f"case {i}: ndim={g.ndim} n={g.n[:g.ndim]} bc={g.bc[:g.ndim]} R={c['R']} {c['scheme']} "
             f"nc={c['nc']} {c['prec']} ell/dx={c['ell'] / max(g.dx[:g.ndim]):.1f} amp={c['amp']}")
    o = oracle.OracleSolver(g, c["R"], c["ell"], c["sigma"], scheme=c["scheme"], flux_corr_terms=c["nc"])
    ref = o.rhs(c["U"])
    s = gw.Solver(g, c["R"], c["ell"], c["sigma"], precision=c["prec"], U0=c["U"], scheme=c["scheme"],
                  flux_corr_terms=c["nc"])
    try:
        got = s.rhs(c["U"])
    finally:
        s.close()
    bound = 32 * EPS[c["prec"]] * local_flux_scale(g, c["U"], c["R"] + 1 + c["nc"])[None]
    if c["scheme"] == "gp-ao":
        rng = np.random.default_rng(11 + i)
        spread = np.zeros_like(ref)
        for _ in range(8):
            Up = c["U"] * (1.0 + EPS[c["prec"]] * rng.uniform(-1.0, 1.0, c["U"].shape))
            spread = np.maximum(spread, np.abs(o.rhs(Up) - ref))
        bound = bound + 4 * spread
    cell = float((np.abs(got - ref) / bound).max())
    announce(f"  worst cell {cell:.3f} of the per-cell bound")
    assert cell <= 1.0


NRUNS = 12


@pytest.mark.parametrize("i", range(NRUNS))
def test_random_configuration_steps_match_oracle(i):
    """20 CFL-limited SSP-RK3 steps through gpweno_run on further random
    configurations: the same step count, relative L1 within 1e-12 (float64) or
    1e-5 (float32), and the per-cell state bound. GP-AO draws run GP-WENO here:
    its conditioning near a vanishing indicator (above) has no state bound."""
    c = draw(100 + i)
    if c["scheme"] == "gp-ao":
        c["scheme"] = "gp-weno"
    g = c["g"]
    # slower flow (a third of the drawn velocities), so that walls do not drive
    # the random data into strong shocks within the run
    rho, vel, p = inputs.cons_to_prim(g, c["U"], 1.4)
    c["U"] = inputs.prim_to_cons(g, rho, [v / 3 for v in vel], p, 1.4)
    tol = 1e-12 if c["prec"] == "fp64" else 1e-5
    announce(f"run {i}: ndim={g.ndim} n={g.n[:g.ndim]} bc={g.bc[:g.ndim]} R={c['R']} {c['scheme']} "
             f"nc={c['nc']} {c['prec']}")
    o = oracle.OracleSolver(g, c["R"], c["ell"], c["sigma"], scheme=c["scheme"], flux_corr_terms=c["nc"])
    Uo = c["U"].copy()
    to, no = o.run(Uo, 1e30, max_steps=20)
    s = gw.Solver(g, c["R"], c["ell"], c["sigma"], precision=c["prec"], U0=c["U"], scheme=c["scheme"],
                  flux_corr_terms=c["nc"])
    try:
        n, t = s.run(1e30, max_steps=20)
        Ug = s.get_state()
    finally:
        s.close()
    assert n == no == 20
    err = float(np.abs(Ug - Uo).sum() / np.abs(Uo).sum())
    cell = state_cell_excess(g, c["U"], Ug, Uo, c["prec"], t, n)
    announce(f"  rel L1 {err:.2e}, worst cell {cell:.3f} of the per-cell bound, t {t:.6e} vs {to:.6e}")
    assert err < tol
    assert cell <= 1.0


def draw_problem(rng, stream):
    """A small random problem for a batch: any dimension, scheme, indicator
    mean, correction terms, boundaries, precision and positivity option."""
    ndim = int(rng.integers(1, 4))
    scheme = ["gp-weno", "weno-js", "weno-gp", "gp-ao"][int(rng.integers(0, 4))]
    R = {"weno-js": int(rng.integers(1, 3)), "gp-ao": int(rng.integers(2, 4))}.get(scheme, int(rng.integers(1, 4)))
    gp_ind = scheme in ("gp-weno", "weno-gp")
    nzm = gp_ind and rng.random() < 0.3
    nc = 3 if gp_ind and not nzm and rng.random() < 0.3 else 2
    prec = ["fp64", "fp32"][int(rng.integers(0, 2))]
    maxn = {1: 90, 2: 36, 3: 14}[ndim]
    n, bc = [], []
    for d in range(ndim):
        if rng.random() < 0.5:
            bc.append((inputs.PERIODIC, inputs.PERIODIC))
            n.append(int(rng.integers(2, maxn + 1)))
        else:
            bc.append(tuple(int(x) for x in rng.choice([inputs.OUTFLOW, inputs.REFLECT], size=2)))
            n.append(int(rng.integers(R + 1 + nc, maxn + 1)))
    h = 1.0 / 64
    hi = [nd * h for nd in n]                      # square cells: one table set per kind
    if ndim == 1:
        g = inputs.grid1d(n[0], 0.0, hi[0], bc)
    elif ndim == 2:
        g = inputs.grid2d(n[0], n[1], (0.0, 0.0), tuple(hi), bc)
    else:
        g = inputs.grid3d(n[0], n[1], n[2], (0.0, 0.0, 0.0), tuple(hi), bc)
    U = inputs.random_smooth(g, seed=int(rng.integers(0, 1 << 30)))
    rho, vel, p = inputs.cons_to_prim(g, U, 1.4)
    U = inputs.prim_to_cons(g, rho, [v / 3 for v in vel], p, 1.4)
    opts = dict(precision=prec, scheme=scheme, nonzero_mean=nzm, flux_corr_terms=nc,
                positivity_fallback=bool(rng.random() < 0.3))
    sigma = (1.8 if scheme == "gp-ao" else 3.0) * h
    return g, U, R, 12 * h, sigma, opts


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_batch_mixes_are_bitwise_single(seed):
    """Random sets of small problems of every kind the batch groups (dimension,
    scheme, indicator mean, correction terms, boundaries, precision) join and
    leave a batch between runs, some before they reach their step limit; every
    problem ends bitwise equal to its own single-problem run of the steps it
    took."""
    rng = np.random.default_rng(500 + seed)
    stream = torch.cuda.Stream()
    b = gw.Batch(stream)
    probs = []          # (solver, (g, U, R, ell, sigma, opts), limit)

    def admit(k, room):
        for _ in range(k):
            g, U, R, ell, sigma, opts = draw_problem(rng, stream)
            limit = int(rng.integers(2, room + 1))
            s = gw.Solver(g, R, ell, sigma, U0=U, stream=stream, **opts)
            s.set_end(1e30, limit)
            probs.append((s, (g, U, R, ell, sigma, opts), limit))

    runs = [6, 5, 7]
    admit(7, sum(runs))
    active = list(range(len(probs)))
    for r, k in enumerate(runs):
        if r > 0:
            # some leave, new ones join with limits that fit the runs left
            active = [j for j in active if rng.random() < 0.6]
            before = len(probs)
            admit(int(rng.integers(2, 5)), sum(runs[r:]))
            active += list(range(before, len(probs)))
        announce(f"mix {seed}, run {r}: {len(active)} problems, "
                 f"{len({(p[1][0].ndim, p[1][2], p[1][5]['precision'], p[1][5]['scheme']) for p in (probs[j] for j in active)})} kinds")
        b.set([probs[j][0] for j in active])
        b.run(k)
    b.status()
    try:
        for s, (g, U, R, ell, sigma, opts), limit in probs:
            done = s.time()[2]
            assert 1 <= done <= limit and not s.failure()[0]
            ref = gw.Solver(g, R, ell, sigma, U0=U, **opts)
            ref.run(1e30, max_steps=done)
            assert ref.time()[2] == done
            assert np.array_equal(s.get_state(), ref.get_state()), (g.n, R, opts)
            ref.close()
    finally:
        b.close()


NBOXES = 10


def riemann_box(i):
    """Random piecewise-constant data: 2^ndim orthants of constant state (rho
    and p in [0.5, 1.5], velocities in [-0.3, 0.3]) on a random grid and
    boundary set, the positivity fallback on."""
    rng = np.random.default_rng(8000 + i)
    c = draw(200 + i)
    if c["scheme"] == "gp-ao":
        c["scheme"] = "gp-weno"
    g = c["g"]
    X = g.mesh()
    q = np.zeros(g.shape, dtype=int)
    for d in range(g.ndim):
        mid = 0.5 * (g.lo[d] + g.hi[d]) + float(rng.uniform(-0.2, 0.2)) * (g.hi[d] - g.lo[d])
        q += (X[d] >= mid).astype(int) << d
    k = 1 << g.ndim
    rho = rng.uniform(0.5, 1.5, k)[q]
    p = rng.uniform(0.5, 1.5, k)[q]
    vel = [rng.uniform(-0.3, 0.3, k)[q] for _ in range(g.ndim)]
    c["U"] = inputs.prim_to_cons(g, rho, vel, p, 1.4)
    return c


@pytest.mark.parametrize("i", range(NBOXES))
def test_random_riemann_data_steps_match_oracle(i):
    """15 CFL steps of random piecewise-constant (Riemann) data on random
    grids and boundaries, positivity fallback on: the same step count and
    relative L1 within 1e-12 (float64) or 1e-5 (float32). No per-cell bound:
    at a jump the nonlinear weights amplify rounding as the flux scale does not
    describe. Closed or periodic boxes also keep their float64 totals."""
    c = riemann_box(i)
    g = c["g"]
    tol = 1e-12 if c["prec"] == "fp64" else 1e-5
    announce(f"riemann {i}: ndim={g.ndim} n={g.n[:g.ndim]} bc={g.bc[:g.ndim]} R={c['R']} {c['scheme']} "
             f"nc={c['nc']} {c['prec']}")
    o = oracle.OracleSolver(g, c["R"], c["ell"], c["sigma"], scheme=c["scheme"], flux_corr_terms=c["nc"],
                            positivity_fallback=True)
    Uo = c["U"].copy()
    to, no = o.run(Uo, 1e30, max_steps=15)
    s = gw.Solver(g, c["R"], c["ell"], c["sigma"], precision=c["prec"], U0=c["U"], scheme=c["scheme"],
                  flux_corr_terms=c["nc"], positivity_fallback=True)
    try:
        tot0 = s.conserved_sums()
        n, t = s.run(1e30, max_steps=15)
        tot1 = s.conserved_sums()
        Ug = s.get_state()
    finally:
        s.close()
    assert n == no == 15
    err = float(np.abs(Ug - Uo).sum() / np.abs(Uo).sum())
    announce(f"  rel L1 {err:.2e}")
    assert err < tol
    closed = all(b[0] in (inputs.PERIODIC, inputs.REFLECT) and b[1] in (inputs.PERIODIC, inputs.REFLECT)
                 for b in g.bc[:g.ndim])
    if closed:
        # mass and energy (and the momentum of periodic axes) stay put up to
        # float64 rounding; a wall exchanges normal momentum with the box
        scale = np.abs(c["U"]).reshape(g.nv, -1).sum(axis=1)
        bound = conserved_totals_bound(g.ncells, n, scale)
        keep = [0, g.nv - 1] + [1 + d for d in range(g.ndim) if g.bc[d][0] == inputs.PERIODIC]
        assert np.all(np.abs(tot1 - tot0)[keep] <= bound[keep]), (tot0, tot1)
