#!/usr/bin/env python3
"""Benchmark of the GP-WENO FD-Prim hot path on one MI355X.

A step is one SSP-RK3 step (CFL time step, three stages, each stage one fused
sweep per direction) of the whole grid. Default workload (the headline line):
the 2D isentropic vortex, 512 x 512 periodic cells on [-5,5]^2, vortex strength
5, gamma = 1.4, GP-R2 with ell = 12 dx, sigma = 3 dx, CFL 0.4, one period t = 10.

Reported (one JSON line):
  value        cell-updates/s per RK stage of the float32-sweep path (float64 state)
  fp64         the same for the all-float64 path
  roofline     the dominant sweep kernel of the headline workload, timed with HIP
               events on its stream; achieved flop rate by the algorithmic count
               of one cell in one direction (a per-cell tally of the path's steps)
  workloads    the Kelvin-Helmholtz (2048 x 1024, GP-R3) and 3D density-wave
               (256^3, GP-R2) workloads: the same timing and roofline, plus the
               HBM rate of every sweep from the committed rocprofv3 counters
  accuracy     relative L1 of both paths against the float64 CPU oracle after the
               full runs (C2 to t = 10, C3 200 steps, C4 wave and vortex 50
               steps), and density L1 against the exact solution
  latency      p50/p99 time-to-solution of full solves (upload, run, download)
  serving      the continuous-batching request loop on a Poisson stream, with a
               budget that does and one that does not make admission wait
  time_to_error the paper's time-to-error comparison of GP-R1/R2/R3, WENO-GP and
               WENO-JS
  cpu_baseline the CPU oracle timed on a bounded sample of the headline workload
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402

METRIC = "cell-updates/sec per RK stage (FP32 vs FP64 at stated L1 err); p50/p99 solve latency"
# MI355X published peaks. The fp32 vector figure assumes packed dual-issue FP32;
# the library is built without packed FP32, so its attainable fp32 vector peak
# is the unpacked 78.6 TFLOP/s (256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz),
# reported beside the published one.
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
PEAK_TFLOPS_UNPACKED = 78.6
PEAK_HBM_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1808_04960_amd", "csrc")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _code_only(text: str) -> str:
    """Source text without comments and whitespace (the sources hold no string
    literal with a comment marker), so that editing a comment does not count as
    a kernel change."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return "".join(text.split())


def kernel_source_hash() -> str:
    """sha256[:16] of the device sources (every .hip file and the kernel headers),
    comments and whitespace excluded."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hip") or name in ("gpweno_sweep.h", "gpweno_kernels.h"):
            with open(os.path.join(CSRC, name), encoding="utf-8") as fh:
                h.update(name.encode() + b"\0" + _code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def flops_per_cell_dir(ndim: int, R: int) -> int:
    """Algorithmic flops of one cell in one direction (FMA = 2, square root and
    division = 1), a per-cell tally of the path's steps in their plain forms:
      eigen quantities 10, projection 10 n (n = 2R+1),
      GP-WENO per characteristic field 4(R+1)^2 (indicators) + 2(R+1)^2(R+2)
        (candidates at both points) + 13(R+1) (weights, combination),
      back-projection 16, HLLC 90, flux correction and difference 9 nv.
    2D R2: 790; 2D R3: 1326; 3D R2: 946. A sweep that finishes an RK stage adds
    4 nv for the stage combination (flops_per_launch)."""
    nv = 2 + ndim
    n = 2 * R + 1
    field = 4 * (R + 1) ** 2 + 2 * (R + 1) ** 2 * (R + 2) + 13 * (R + 1)
    return 10 + 10 * n + nv * field + 16 + 90 + 9 * nv


def flops_per_cell_dir_evaluated(ndim: int, R: int, fp64: bool = False) -> int:
    """The flops of the forms the sweep evaluates (the indicator on mirrored sums
    and differences, candidates pre-multiplied by their linear weights, the
    one-sided HLLC flux, the correction gathered by neighbour distance):
      cons->prim 3 ndim + 3, eigen quantities 8, projection 6n,
      per field (R+1) b_R + 2(R+1)(2R+1) + W_R (b = 10/15/24; W_R: float32
      11(R+1) + 2, float64 (R+1) + p_R + 8R + 8 with p = 0/3/6),
      back-projection 14, HLLC 43 + 5(ndim-1) + 3 nv, correction and difference 9 nv.
    Fewer than flops_per_cell_dir: the same results from cheaper forms."""
    nv = 2 + ndim
    n = 2 * R + 1
    beta_window = {1: 10, 2: 15, 3: 24}[R]
    weights = (R + 1) + {1: 0, 2: 3, 3: 6}[R] + 8 * R + 8 if fp64 else 11 * (R + 1) + 2
    weno = (R + 1) * beta_window + 2 * (R + 1) * (2 * R + 1) + weights
    hllc = 43 + 5 * (ndim - 1) + 3 * nv
    return (3 * ndim + 3) + 8 + 6 * n + nv * weno + 14 + hllc + 9 * nv


def flops_per_launch(ndim, R, ncell, fin):
    return (flops_per_cell_dir(ndim, R) + (4 * (2 + ndim) if fin else 0)) * ncell


def algorithmic_bytes_per_step(ndim, ncell):
    """Algorithmic bytes: per cell-update (one cell through one RK
    stage, all directions) (8/3) nv s with s = 8 (float64 state): read the stage
    state, write the next, and read U^n in stages 2 and 3. Three per step."""
    return 3 * ncell * (8.0 / 3.0) * (2 + ndim) * 8


WORKLOADS = {
    "vortex2d": dict(desc="2D isentropic vortex, 512x512 periodic on [-5,5]^2, strength 5, gamma 1.4, "
                          "GP-R2 (ell=12dx, sigma=3dx), SSP-RK3 CFL 0.4, t=10",
                     make=lambda: inputs.isentropic_vortex_2d(512), R=2, t_final=10.0, tag="vortex2d_512_R2",
                     ref="vortex2d_512"),
    "sine1d": dict(desc="1D sine density wave, N=128 periodic on [0,1], GP-R2, CFL 0.4, t=1",
                   make=lambda: inputs.sine_wave_1d(128), R=2, t_final=1.0, tag="sine1d_128_R2"),
    "kh2d": dict(desc="2D Kelvin-Helmholtz, 2048x1024 periodic on [0,2]x[0,1], rho 2/1, u +-0.5, p 2.5, seeded 1% "
                      "velocity noise, GP-R3 (ell=12dx, sigma=3dx), CFL 0.4, 200 steps",
                 make=lambda: inputs.kelvin_helmholtz_2d(2048, 1024), R=3, t_final=None, tag="kh2d_2048x1024_R3",
                 full_steps=200),
    "wave3d": dict(desc="3D density wave, 256^3 periodic on [0,1]^3, GP-R2 (ell=12dx, sigma=3dx), CFL 0.4, 50 steps",
                   make=lambda: inputs.density_wave_3d(256), R=2, t_final=None, tag="wave3d_256_R2", full_steps=50,
                   ref="wave3d_256"),
    "vortex3d": dict(desc="3D isentropic vortex (w=0), 256^3 periodic on [-5,5]^3, GP-R2, CFL 0.4, 50 steps",
                     make=lambda: inputs.isentropic_vortex_3d(256), R=2, t_final=None, tag="vortex3d_256_R2",
                     full_steps=50, ref="vortex3d_256"),
    # the paper's 3D explosion (Sec. 7, Eq. (3d-exp)) at its resolution and CFL;
    # outflow boundaries, so the sweeps run the general-boundary kernels. The
    # solve reaches t = 0.25 in 276 steps; the timed runs stay inside that span
    # (max_steps), since far beyond it, after the blast has left the box, the
    # scheme (which has no positivity limiter) meets a non-physical state.
    "explosion3d": dict(desc="3D explosion, 128^3 on [-1,1]^3 with outflow boundaries, GP-R2 (ell=12dx, sigma=3dx), "
                             "SSP-RK3 CFL 0.3, t=0.25",
                        make=lambda: inputs.explosion(3, 128), R=2, t_final=0.25, tag="explosion3d_128_R2", cfl=0.3,
                        bcg=True, exact=False, max_steps=260),
}

SERVING_DESC = ("Poisson stream (seed 0, mean 20 req/s) of independent 2D Euler problems, grids uniform from "
                "{64^2..1024^2}, R in {1,2,3}, 100-500 steps, half isentropic vortex / half random four-quadrant "
                "Riemann data, FIFO admission by HBM footprint (64 slots), fp32 sweep arithmetic")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_serving(count, budget, slots, steps_per_tick, rate=20.0):
    """Replays the serving stream through the continuous-batching server."""
    from paper_1808_04960_amd.serve import GpuExecutor, Server

    reqs = inputs.serving_stream(count=count, rate=rate, seed=0)
    for r in reqs:
        r.cache_state()
    offered = sum(3.0 * r.steps * r.cells for r in reqs)
    ex = GpuExecutor("fp32")
    # warm the kernels and the allocator on a short private stream of the same mix
    warm = inputs.serving_stream(count=12, rate=1e6, seed=99, steps=(2, 4))
    Server(ex, hbm_budget=budget, max_slots=slots, steps_per_tick=steps_per_tick).run(warm)
    rep = Server(ex, hbm_budget=budget, max_slots=slots, steps_per_tick=steps_per_tick).run(reqs, keep_results=True)
    s = rep.summary()
    s["offered_cell_updates"] = offered
    s["offered_rate_req_s"] = rate
    s["hbm_budget_bytes"] = budget
    s["arrival_span_s"] = reqs[-1].arrival - reqs[0].arrival
    waits = [j.admitted - j.req.arrival for j in rep.jobs if j.status == "done"]
    s["admission_wait_p50_ms"] = float(np.percentile(waits, 50) * 1e3)
    s["admission_wait_p99_ms"] = float(np.percentile(waits, 99) * 1e3)
    s["what"] = ("latency = arrival to result on the host; admission wait = arrival to admission; "
                 "cell_updates_per_s = work / (last completion - first arrival)")
    for j in rep.jobs:
        j.result = None
    ex.close()
    log(f"serving (budget {budget >> 20} MiB, {rate:g} req/s): {s['completed']}/{s['requests']} done, "
        f"p50 {s['p50_ms']:.1f} ms, p99 {s['p99_ms']:.1f} ms, admission wait p99 {s['admission_wait_p99_ms']:.1f} ms, "
        f"{s['cell_updates_per_s']:.3e} cell-updates/s, peak {s['peak_active']} active, "
        f"{s['peak_resident_bytes'] >> 20} MiB resident")
    return s


TTE_DESC = ("2D isentropic vortex on [0,20]^2 (strength 5, background rho = u = v = p = 1, gamma 1.4), one "
            "period t = 20, ell = 1.2, sigma = 3 dx, CFL 0.4 without time-step reduction, SSP-RK3, float64 sweeps; "
            "L1 = 100 x mean |rho - rho(t=0)|")
TTE_CASES = (("weno-js", 2, (64, 96, 128, 192)), ("weno-gp", 2, (64, 96, 128, 192)),
             ("gp-weno", 1, (192, 256, 384, 512)), ("gp-weno", 2, (48, 64, 96, 128)),
             ("gp-weno", 3, (48, 64, 96, 128)))


def _interp_time(points, target):
    """Time at which the L1 error reaches target, interpolated log-log between the
    two grids that bracket it; None if no pair does."""
    pts = sorted(points, key=lambda p: -p[0])
    for (e0, t0), (e1, t1) in zip(pts, pts[1:]):
        if e0 >= target >= e1 and e0 > e1:
            f = math.log(e0 / target) / math.log(e0 / e1)
            return t0 * (t1 / t0) ** f
    return None


def time_to_error(target, cells_per_batch=1 << 20, max_copies=64):
    """The shape of the paper's time-to-error study (Sec. 6.2, Fig. (vortex_timing),
    Table (performace-time-to-error)) on the GPU. For each scheme and grid:
      single  -- wall time of one solve to t = 20 (state resident, graph replays);
      batched -- wall time per problem when copies of the problem fill the GPU
                 through the batched path (about cells_per_batch cells in flight);
    each interpolated log-log to the target L1 error, and divided by WENO-JS's
    (the paper's normaliser) and by WENO-GP's (the same polynomial interpolation
    with the GP indicators, whose errors match the paper's printed column)."""
    import torch

    import paper_1808_04960_amd as gw

    out = {"workload": TTE_DESC, "target_l1": target, "schemes": {}}
    for scheme, R, sizes in TTE_CASES:
        name = {"weno-js": "WENO-JS", "weno-gp": "WENO-GP"}.get(scheme, f"GP-R{R}")
        rows = []
        for n in sizes:
            g, U = inputs.isentropic_vortex_2d(n, lo=0.0, hi=20.0)
            dx = g.dx[0]
            s = gw.Solver(g, R, 1.2, 3 * dx, precision="fp64", U0=U, scheme=scheme)
            s.run(20.0, max_steps=40)                      # graph capture, clocks up
            s.set_state(U)
            s.synchronize()
            t0 = time.perf_counter()
            nst, tf = s.run(20.0)
            single = time.perf_counter() - t0
            Ug = s.get_state()
            err = 100.0 * float(np.mean(np.abs(Ug[0] - U[0])))
            s.close()
            copies = max(1, min(max_copies, cells_per_batch // (n * n)))
            stream = torch.cuda.Stream()
            members = []
            for _ in range(copies):
                m = gw.Solver(g, R, 1.2, 3 * dx, precision="fp64", U0=U, scheme=scheme, stream=stream)
                m.set_end(20.0, -1)
                members.append(m)
            b = gw.Batch(stream)
            b.set(members)
            stream.synchronize()
            t0 = time.perf_counter()
            b.run(nst)
            _, _, ns, er = b.status()
            batched = (time.perf_counter() - t0) / copies
            assert (ns == nst).all() and not er.any()
            same = bool(np.array_equal(members[-1].get_state(), Ug))
            b.close()
            for m in members:
                m.close()
            del members
            torch.cuda.empty_cache()
            rows.append({"n": n, "steps": nst, "l1": err, "single_s": single, "copies": copies,
                         "batched_s_per_problem": batched, "batch_bitwise_equal_single": same})
            log(f"time-to-error {name} n={n}: {nst} steps, L1 {err:.3e}, single {single * 1e3:.1f} ms, "
                f"batched {batched * 1e3:.2f} ms/problem ({copies} copies)")
        out["schemes"][name] = {
            "runs": rows,
            "single_s": _interp_time([(r["l1"], r["single_s"]) for r in rows], target),
            "batched_s": _interp_time([(r["l1"], r["batched_s_per_problem"]) for r in rows], target),
            "cell_updates": _interp_time([(r["l1"], 3.0 * r["steps"] * r["n"] ** 2) for r in rows], target),
        }
    for norm in ("WENO-JS", "WENO-GP"):
        ref = out["schemes"][norm]
        key = norm.lower().replace("-", "_")
        for v in out["schemes"].values():
            for k in ("single_s", "batched_s", "cell_updates"):
                v[f"{k}_rel_{key}"] = v[k] / ref[k] if v[k] and ref[k] else None
    out["paper_relative_time"] = {"GP-R1": 35.81, "GP-R2": 0.43, "GP-R3": 0.22, "WENO-JS": 1.0,
                                  "what": "CPU time on 4 cores with RK4, ell = 1.2 (the paper's table)"}
    out["note"] = ("WENO-JS errors here are 2-3x the paper's printed WENO-JS column (which variant the paper ran is "
                   "not stated), while WENO-GP matches its column within 1.5 %: ratios to WENO-GP are the pinned ones")
    return out


def profile_entries():
    """Committed rocprofv3 counter figures per (kernel, workload): HBM bytes fetched
    and written per launch (profiles/traffic.txt) and VALU-busy fraction
    (profiles/valu_busy.txt), with the device-source hash they were taken at."""
    out = {}
    for fname, cols in (("traffic.txt", ("fetch", "write")), ("valu_busy.txt", ("valu_busy",))):
        path = os.path.join(ROOT, "profiles", fname)
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            for line in fh:
                line = line.strip()
                if not line or line.startswith("#"):
                    continue
                parts = line.split()
                key = (parts[0], parts[1], parts[-1])
                rec = out.setdefault(key, {})
                for i, c in enumerate(cols):
                    rec[c] = float(parts[2 + i])
    return out


def counters_for(kernel_name, tag, entries, sha):
    return entries.get((kernel_name.replace(" ", ""), sha, tag), {})


def kernel_symbol(ndim, d, R, real, fin, bcg=False):
    """rocprofv3 name of a sweep: template arguments ndim, direction, R, real type,
    finishes the stage, indicator kind (0: GP), general boundaries, flux
    correction terms."""
    return (f"sweep_kernel<{ndim}, {d}, {R}, {real}, {'true' if fin else 'false'}, 0, "
            f"{'true' if bcg else 'false'}, 2>")


KERNEL_TIMING_HOLD_S = 0.05   # stream hold while the host enqueues the kernel-timing phase


def phase_reps(reps, span_s, phase_s):
    """Repeats per launch of the second kernel-timing pass: the first pass of
    `reps` repeats took span_s seconds; a pass shorter than phase_s is scaled
    up to fill it, by at most 1000 times (None: the first pass is long
    enough)."""
    if span_s >= phase_s:
        return None
    return int(math.ceil(reps * min(1000.0, phase_s / max(span_s, 1e-9))))


def time_workload(name, W, grid, U0, steps, warmup, kernel_reps, kernel_phase_s=0.0):
    """Per precision: every launch of the step sequence timed back to back with
    HIP events on the solver's stream, then the warm-up and the timed
    graph-replayed steps. The kernel timing comes first (after one step that
    captures the step graphs): a pass of kernel_reps repeats per launch, then,
    if that pass took less than kernel_phase_s, a second pass with the repeats
    scaled up to fill it, whose times are the ones reported. The GPU's clocks
    follow its load: a pass of a few milliseconds times the 512^2 sweeps about
    5 % slow (9.03 against 8.6 us), and a 20-step window right after it runs
    56.7-57.2 us per step against 55.0 after a 0.2 s phase (53 us in a long
    run). The timed window is exactly `steps` steps either way.
    Returns (solvers, wall seconds per precision, per-kernel (mean us, launches per step))."""
    import torch

    import paper_1808_04960_amd as gw

    R = W["R"]
    dx = grid.dx[0]
    ncell = grid.ncells
    t_run = 1e9  # timing runs never reach their end time
    nk = 3 * grid.ndim
    solvers, timing, kern = {}, {}, {}
    for prec in ("fp32", "fp64"):
        s = gw.Solver(grid, R, 12 * dx, 3 * dx, precision=prec, cfl=W.get("cfl", 0.4), U0=U0)
        solvers[prec] = s
        U0_dev = s.state.clone()   # the initial state on the device (restores without host uploads)
        s.run(t_run, max_steps=1)  # captures the step graphs
        s.synchronize()
        # per-kernel launch durations: each launch of the step sequence
        # (gpweno_step_kernel k) repeated back to back between two HIP events on
        # the solver's stream. Every launch reads and writes the same buffers as
        # in a step, so a repeat does the same work. A bounded spin holds the
        # stream while the host enqueues the phase; the phase then runs back to
        # back, without launch gaps and without idle time up to the timed
        # window. (Under a profiler that slows every launch on the host, the
        # launches of small grids are no longer back to back: compare profiled
        # kernel durations, not profiled event times.)
        real = "float" if prec == "fp32" else "double"

        def kernel_pass(reps):
            with torch.cuda.stream(s.stream):
                torch.cuda._sleep(int(2.4e9 * KERNEL_TIMING_HOLD_S))
            t_enq = time.perf_counter()
            marks = []
            for k in range(nk):
                s.set_state(U0_dev)
                s.step(t_run)  # sets the end time and lifts the step limit
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s.stream)
                for _ in range(reps):
                    s.step_kernel(k)
                e1.record(s.stream)
                marks.append((k, e0, e1))
            t_enq = time.perf_counter() - t_enq
            s.synchronize()
            if t_enq > KERNEL_TIMING_HOLD_S:
                # either the host waited for queue space (the queue stayed full:
                # no gaps) or it enqueued slower than the GPU ran (gaps, then
                # timed too)
                log(f"note: enqueueing the kernel timing took {t_enq * 1e3:.0f} ms, more than the "
                    f"{KERNEL_TIMING_HOLD_S * 1e3:.0f} ms hold")
            return marks

        reps = kernel_reps
        marks = kernel_pass(reps)
        span = sum(e0.elapsed_time(e1) for _, e0, e1 in marks) * 1e-3
        more = phase_reps(reps, span, kernel_phase_s)
        if more is not None:
            reps = more
            marks = kernel_pass(reps)
            log(f"  kernel timing: {reps} repeats per launch (the {kernel_reps}-repeat pass took "
                f"{span * 1e3:.1f} ms)")
        per_sym = {}
        for k, e0, e1 in marks:
            d = grid.ndim - 1 - k % grid.ndim   # sweeps of a stage run z, y, x; x finishes it
            sym = kernel_symbol(grid.ndim, d, R, real, d == 0, W.get("bcg", False))
            per_sym.setdefault(sym, []).append(e0.elapsed_time(e1) / reps * 1e-3)
        for sym, ts in per_sym.items():
            kern[(prec, sym)] = (float(np.mean(ts)), len(ts))
            log(f"  {sym}: {np.mean(ts) * 1e6:.2f} us per launch, {len(ts)} per step")
        # the warm-up and the timed steps, from the initial state
        s.set_state(U0_dev)
        s.run(t_run, max_steps=warmup)
        s.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n, _ = s.run(t_run, max_steps=steps)
        s.synchronize()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert n == steps
        timing[prec] = el
        del U0_dev
        log(f"{name} {prec}: {steps} steps in {el * 1e3:.2f} ms -> {ncell * 3 * steps / el:.4e} cell-updates/s")
    return solvers, timing, kern


def limiter(valu_busy, hbm_frac):
    """What the counters say bounds a sweep: VALU issue when the VALUs issue at
    least 3/4 of the kernel's time, HBM when the counted traffic runs at 60 %
    of the peak or more, else latency (waits that computation does not cover:
    on a small grid, where every wave of a launch is resident at once, the
    launch's start and end)."""
    if valu_busy is None:
        return None
    if valu_busy >= 0.75:
        return f"VALU issue (busy {valu_busy:.2f})"
    if hbm_frac is not None and hbm_frac >= 0.6:
        return f"HBM ({hbm_frac:.2f} of peak)"
    return f"latency (VALU busy {valu_busy:.2f}, HBM {hbm_frac or 0:.2f} of peak)"


def roofline_of(W, grid, timing, kern, steps, prec, entries, sha):
    """Roofline of the dominant kernel (largest time per step) of one precision,
    and every sweep's rates."""
    ndim, R, ncell = grid.ndim, W["R"], grid.ncells
    syms = [k[1] for k in kern if k[0] == prec]
    dom = max(syms, key=lambda sym: kern[(prec, sym)][0] * kern[(prec, sym)][1])
    per = {}
    for sym in syms:
        t, cnt = kern[(prec, sym)]
        targs = sym[sym.index("<") + 1:sym.rindex(">")].split(", ")
        fin = targs[4] == "true"
        fl = flops_per_launch(ndim, R, ncell, fin)
        c = counters_for(sym, W["tag"], entries, sha)
        traffic = (c["fetch"] + c["write"]) if "fetch" in c else None
        per[sym] = {"avg_launch_us": t * 1e6, "launches_per_step": cnt, "flops_per_launch": fl,
                    "achieved_tflops": fl / t / 1e12,
                    "frac_of_published_peak": fl / t / 1e12 / PEAK_TFLOPS[prec],
                    "frac_of_unpacked_peak": fl / t / 1e12 / PEAK_TFLOPS_UNPACKED,
                    "hbm_bytes_per_launch": traffic,
                    "hbm_gbs": traffic / t / 1e9 if traffic else None,
                    "hbm_frac": traffic / t / 1e9 / PEAK_HBM_GBS if traffic else None,
                    "valu_busy": c.get("valu_busy")}
        per[sym]["limited_by"] = limiter(per[sym]["valu_busy"], per[sym]["hbm_frac"])
    p = per[dom]
    step_s = timing[prec] / steps
    alg_bytes = algorithmic_bytes_per_step(ndim, ncell)
    return {"bound": "alu", "achieved": p["achieved_tflops"], "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
            "frac": p["frac_of_published_peak"], "traffic": p["hbm_bytes_per_launch"], "kernel": dom,
            "avg_launch_us": p["avg_launch_us"], "flops_per_launch": p["flops_per_launch"],
            "flops_per_cell_dir": flops_per_cell_dir(ndim, R),
            "flops_per_cell_dir_evaluated_form": flops_per_cell_dir_evaluated(ndim, R, prec == "fp64"),
            "frac_of_unpacked_peak": p["frac_of_unpacked_peak"], "peak_unpacked": PEAK_TFLOPS_UNPACKED,
            "valu_busy": p["valu_busy"], "hbm_gbs": p["hbm_gbs"], "hbm_frac": p["hbm_frac"],
            "limited_by": p["limited_by"],
            "algorithmic_bytes_per_step": alg_bytes,
            "algorithmic_hbm_gbs": alg_bytes / step_s / 1e9,
            "algorithmic_hbm_frac": alg_bytes / step_s / 1e9 / PEAK_HBM_GBS,
            "kernel_sum_us_per_step": sum(v["avg_launch_us"] * v["launches_per_step"] for v in per.values()),
            "kernels": per}


def full_length_accuracy(name, W, grid, U0, solvers, run_c3_oracle):
    """Relative L1 of both paths against the oracle after the workload's full run
    (stored oracle states for C2 and C4; the C3 oracle runs here on the host)."""
    R = W["R"]
    t_final = W["t_final"] if W["t_final"] is not None else 1e9
    max_steps = W.get("full_steps", -1)
    out = {}
    ref = None
    if "ref" in W:
        with np.load(os.path.join(GOLDEN, f"oracle_{W['ref']}.npz"), allow_pickle=False) as z:
            ref = {k: z[k] for k in z.files}
    elif name == "kh2d" and run_c3_oracle:
        import oracle

        dx = grid.dx[0]
        t0 = time.perf_counter()
        Uo = U0.copy()
        t_o, n_o = oracle.OracleSolver(grid, R, 12 * dx, 3 * dx).run(Uo, t_final, max_steps=max_steps)
        log(f"{name}: oracle {n_o} steps in {time.perf_counter() - t0:.0f} s on {oracle.threads()} threads")
        ref = {"U": Uo, "t": t_o, "nsteps": n_o, "form": "full"}
    if ref is None:
        return None
    for prec in ("fp32", "fp64"):
        s = solvers[prec]
        s.set_state(U0)
        n, t = s.run(t_final, max_steps=max_steps)
        Ug = s.get_state()
        if "f" in ref:       # wave: a function of (i+j+k) mod n, plus its stored deviation
            N = grid.n[0]
            idx = (np.arange(N)[:, None, None] + np.arange(N)[None, :, None] + np.arange(N)[None, None, :]) % N
            num = sum(float(np.abs(Ug[k] - ref["f"][k][idx]).sum()) for k in range(grid.nv))
            err = (num + float(ref["dev_l1"])) / float(ref["norm_l1"])
        elif "slice" in ref:  # uniform in z
            Uref = ref["slice"][:, None]
            err = float(np.abs(Ug - Uref).sum() / (np.abs(Uref).sum() * Ug.shape[1]))
        else:
            err = float(np.abs(Ug - ref["U"]).sum() / np.abs(ref["U"]).sum())
        out[f"{prec}_rel_l1_vs_oracle"] = err
        out[f"{prec}_steps"] = int(n)
        out["oracle_steps"] = int(ref["nsteps"])
        assert n == int(ref["nsteps"]), (name, prec, n, int(ref["nsteps"]))
        if W.get("exact", True) and W["t_final"] is not None:
            out[f"{prec}_density_l1_vs_exact"] = float(np.mean(np.abs(Ug[0] - U0[0])))
        log(f"{name} {prec}: {n} steps to t={t:.4g}, rel L1 vs oracle {err:.3e}")
    return out


# ---------------------------------------------------------------------------
# Summaries of rocprofv3 output (profiles/)
# ---------------------------------------------------------------------------
PROFILE_TAGS = {(2, 2): "vortex2d_512_R2", (2, 3): "kh2d_2048x1024_R3", (3, 2): "wave3d_256_R2",
                (1, 2): "sine1d_128_R2"}
PROFILE_CELLS = {"vortex2d_512_R2": 512 * 512, "kh2d_2048x1024_R3": 2048 * 1024, "wave3d_256_R2": 256 ** 3,
                 "sine1d_128_R2": 128}
COPY_BYTES = 1 << 30   # the --copy-probe copy


def _short_name(name):
    name = name.strip('"')
    if name.startswith("void "):
        name = name[5:]
    name = name.split("(")[0]
    return name[name.index("sweep_kernel"):] if "sweep_kernel" in name else name


def _read_csv(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _counters(raw):
    """Mean over dispatches of every counter, per kernel, from run_counter_collection.csv."""
    sums, counts = {}, {}
    for row in _read_csv(raw):
        k = (_short_name(row["Kernel_Name"]), row["Counter_Name"])
        sums[k] = sums.get(k, 0.0) + float(row["Counter_Value"])
        counts[k] = counts.get(k, 0) + 1
    out = {}
    for (kern, ctr), v in sums.items():
        out.setdefault(kern, {})[ctr] = v / counts[(kern, ctr)]
    return out


def _copy_calibration(raw, counter):
    """Value of the counter for the --copy-probe copy (the largest copyBuffer dispatch)."""
    vals = [float(r["Counter_Value"]) for r in _read_csv(raw)
            if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == counter]
    return max(vals) if vals else None


def _trace_split(path, min_run):
    """Per sweep kernel, the mean duration (us) of its back-to-back launches
    (runs of at least min_run identical consecutive dispatches: the benchmark's
    HIP-event timing) and of its launches inside the replayed step sequence,
    with their counts, from a rocprofv3 kernel trace."""
    rows = sorted(_read_csv(path), key=lambda r: int(r["Start_Timestamp"]))
    seq = [(_short_name(r["Kernel_Name"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
           for r in rows]
    out = {}
    i = 0
    while i < len(seq):
        j = i
        while j < len(seq) and seq[j][0] == seq[i][0]:
            j += 1
        name = seq[i][0]
        if name.startswith("sweep_kernel"):
            slot = out.setdefault(name, {"b2b": [], "seq": []})
            slot["b2b" if j - i >= min_run else "seq"].extend(d for _, d in seq[i:j])
        i = j
    return {k: {w: (len(v[w]), sum(v[w]) / len(v[w]) if v[w] else None) for w in v} for k, v in out.items()}


def summarize_profiles(raw_dir, out_dir, command, stats_command=None, kernel_reps=100):
    """Writes profiles/ summaries from the rocprofv3 passes in raw_dir
    (prof_stats: --kernel-trace --stats of stats_command; prof_fetch / prof_write:
    --pmc FETCH_SIZE / WRITE_SIZE; prof_busy, prof_mixf, prof_mixo: the SQ counter
    sets, all of command)."""
    sha = kernel_source_hash()
    stats_command = stats_command or command
    stats = {}
    for row in _read_csv(os.path.join(raw_dir, "prof_stats", "run_kernel_stats.csv")):
        n = _short_name(row["Name"])
        if n.startswith("sweep_kernel"):
            stats[n] = (int(row["Calls"]), float(row["AverageNs"]) / 1e3, float(row["MinNs"]) / 1e3,
                        float(row["MaxNs"]) / 1e3, float(row["TotalDurationNs"]) / 1e6)
    trace = os.path.join(raw_dir, "prof_stats", "run_kernel_trace.csv")
    split = _trace_split(trace, min(kernel_reps, 4)) if os.path.exists(trace) else {}

    def launch_us(kern):
        """The duration the benchmark's roofline uses: the back-to-back mean."""
        b = split.get(kern, {}).get("b2b", (0, None))
        return b[1] if b[1] else stats[kern][1]
    ctr = {}
    for pas in ("fetch", "write", "busy", "mixf", "mixo"):
        path = os.path.join(raw_dir, f"prof_{pas}", "run_counter_collection.csv")
        if os.path.exists(path):
            for k, v in _counters(path).items():
                ctr.setdefault(k, {}).update(v)
    fetch_cal = _copy_calibration(os.path.join(raw_dir, "prof_fetch", "run_counter_collection.csv"), "FETCH_SIZE")
    write_cal = _copy_calibration(os.path.join(raw_dir, "prof_write", "run_counter_collection.csv"), "WRITE_SIZE")
    f_scale = COPY_BYTES / (fetch_cal * 1024) if fetch_cal else None
    w_scale = COPY_BYTES / (write_cal * 1024) if write_cal else None

    def targs(kern):
        return kern[kern.index("<") + 1:kern.rindex(">")].split(", ")

    by_tag = {}
    for kern in stats:
        a = targs(kern)
        by_tag.setdefault(PROFILE_TAGS.get((int(a[0]), int(a[2])), "other"), []).append(kern)
    head = (f"# commands (one MI355X, repository root, TMPDIR=/tmp):\n"
            f"#   rocprofv3 --kernel-trace --stats -d <dir> -o run --output-format csv -- python3 bench.py "
            f"{stats_command}\n"
            f"#   rocprofv3 <pass> -d <dir> -o run --output-format csv -- python3 bench.py {command}\n"
            f"#   passes: --pmc FETCH_SIZE | --pmc WRITE_SIZE |\n"
            f"#     --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES "
            f"SQ_WAVE_CYCLES GRBM_GUI_ACTIVE |\n"
            f"#     --pmc SQ_INSTS_VALU_{{ADD,MUL,FMA,TRANS}}_{{F32,F64}} |\n"
            f"#     --pmc SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64 SQ_INSTS_VALU_CVT SQ_INSTS_VALU_FLOPS_FP32 "
            f"SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_LDS_BANK_CONFLICT\n"
            f"#   summarised by: python3 bench.py --summarize-profiles <dir>\n"
            f"# device sources sha256[:16] = {sha} (bench.kernel_source_hash)\n")
    traffic_lines, busy_lines = [], []
    for tag, kerns in sorted(by_tag.items()):
        kerns.sort(key=lambda k: -stats[k][4])
        with open(os.path.join(out_dir, f"kernel_stats_{tag}.txt"), "w") as fh:
            fh.write(f"# rocprofv3 kernel statistics: GP-WENO sweeps, {tag}\n#\n" + head)
            fh.write("# The stats run is the benchmark's timing (K = 20, W = 5) with its other legs off (no CPU\n"
                     "# baseline, latency solves, serving, time-to-error or full-length oracle runs, whose many\n"
                     "# launches are not timed kernels). It holds fp32 and fp64 solvers: the warm-up and timed\n"
                     "# graph-replayed steps, and the back-to-back launches of every kernel of the step sequence\n"
                     "# that bench's HIP events time (its kernel-timing phase: a 100-repeat pass, then one\n"
                     "# scaled to about 0.2 s, whose times bench reports). b2b_us is the mean over all those\n"
                     "# back-to-back launches (what bench's roofline divides by), seq_us the mean inside the\n"
                     "# replayed steps, where a y sweep follows a finishing sweep. sweep_kernel<ndim, dir, R,\n"
                     "# Real, finishes-an-RK-stage, indicator kind, general boundaries, flux-correction terms>;\n"
                     "# the sweeps of a stage run z, y, x and the x sweep finishes it.\n#\n")
            fh.write(f"{'kernel':62s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} "
                     f"{'total_ms':>9s} {'b2b_n':>6s} {'b2b_us':>9s} {'seq_n':>6s} {'seq_us':>9s}\n")
            for k in kerns:
                c, av, mn, mx, tot = stats[k]
                sp = split.get(k, {})
                bn, bu = sp.get("b2b", (0, None))
                qn, qu = sp.get("seq", (0, None))
                fh.write(f"{k:62s} {c:6d} {av:9.2f} {mn:9.2f} {mx:9.2f} {tot:9.3f} {bn:6d} "
                         f"{(bu or float('nan')):9.2f} {qn:6d} {(qu or float('nan')):9.2f}\n")
        with open(os.path.join(out_dir, f"counters_{tag}.txt"), "w") as fh:
            fh.write(f"# rocprofv3 --pmc counters per dispatch (mean over dispatches), {tag}\n#\n" + head)
            fh.write(f"# calibration: a 1 GiB device copy (__amd_rocclr_copyBuffer) reads FETCH_SIZE {fetch_cal} KiB "
                     f"and WRITE_SIZE {write_cal} KiB per dispatch,\n# so FETCH_SIZE is scaled by "
                     f"{f_scale:.3f} and WRITE_SIZE by {w_scale:.3f}.\n"
                     "# derived: hbm_bytes = calibrated fetch + write; valu_busy = SQ_INSTS_VALU x 4 cycles /\n"
                     "# (1024 SIMDs x duration x 2.4 GHz), with the back-to-back duration of kernel_stats_<workload>\n"
                     "# (b2b_us). The instruction classes and SQ_INSTS_VALU_FLOPS_* are wave-level counts (one per\n"
                     "# wave instruction; FLOPS_* count an FMA as 2 per lane), so hw_flops_per_lane_instr =\n"
                     "# (FLOPS_FP32 + FLOPS_FP64) / SQ_INSTS_VALU, and alg_flops_per_lane_instr = the launch's\n"
                     "# algorithmic flops (bench.flops_per_launch) / (64 SQ_INSTS_VALU).\n#\n")
            for k in kerns:
                cv = ctr.get(k, {})
                av_us = launch_us(k)
                fh.write(f"{k}\n")
                for name in sorted(cv):
                    fh.write(f"    {name:32s} {cv[name]:18.1f}\n")
                fb = cv.get("FETCH_SIZE", 0.0) * 1024 * (f_scale or 0)
                wb = cv.get("WRITE_SIZE", 0.0) * 1024 * (w_scale or 0)
                vi = cv.get("SQ_INSTS_VALU")
                busy = vi * 4 / (1024 * av_us * 1e-6 * 2.4e9) if vi else None
                flops = cv.get("SQ_INSTS_VALU_FLOPS_FP32", 0.0) + cv.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0)
                fh.write(f"    {'hbm_bytes':32s} {fb + wb:18.1f}   ({(fb + wb) / (av_us * 1e-6) / 1e9:.0f} GB/s "
                         f"at {av_us:.2f} us)\n")
                if busy is not None:
                    fh.write(f"    {'valu_busy':32s} {busy:18.3f}\n")
                    fh.write(f"    {'hw_flops_per_lane_instr':32s} {flops / vi:18.3f}\n")
                    a = targs(k)
                    if tag in PROFILE_CELLS:
                        alg = flops_per_launch(int(a[0]), int(a[2]), PROFILE_CELLS[tag], a[4] == "true")
                        fh.write(f"    {'alg_flops_per_lane_instr':32s} {alg / (64 * vi):18.3f}\n")
                    busy_lines.append(f"{k.replace(' ', '')} {sha} {busy:.4f} {tag}")
                if fb:
                    traffic_lines.append(f"{k.replace(' ', '')} {sha} {fb:.0f} {wb:.0f} {tag}")
    with open(os.path.join(out_dir, "traffic.txt"), "w") as fh:
        fh.write("# HBM traffic per launch of each sweep kernel, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE\n"
                 "# (see counters_<workload>.txt for the commands and the copy-kernel calibration).\n"
                 "# columns: kernel  kernel-source-sha256[:16]  bytes-fetched  bytes-written  workload\n"
                 "# bench.py reports these only while the kernel source still has the listed hash.\n")
        fh.write("\n".join(sorted(traffic_lines)) + "\n")
    with open(os.path.join(out_dir, "valu_busy.txt"), "w") as fh:
        fh.write("# VALU-busy fraction per launch of each sweep kernel: SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x\n"
                 "# back-to-back duration x 2.4 GHz), from the counters_<workload>.txt passes.\n"
                 "# columns: kernel  kernel-source-sha256[:16]  valu_busy  workload\n")
        fh.write("\n".join(sorted(busy_lines)) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="vortex2d", choices=sorted(WORKLOADS) + ["serving"])
    ap.add_argument("--solves", type=int, default=5, help="full solves for the latency percentiles")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="oracle sample budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=100, help="back-to-back launches per timed kernel")
    ap.add_argument("--kernel-phase-ms", type=float, default=200.0,
                    help="minimum length of the kernel-timing phase: a pass of --kernel-reps repeats that takes "
                         "less is followed by one with the repeats scaled up to this length (0: one pass)")
    ap.add_argument("--serving-requests", type=int, default=200, help="requests of the serving stream (0: skip)")
    ap.add_argument("--no-time-to-error", action="store_true", help="skip the time-to-error study")
    ap.add_argument("--no-extra-workloads", action="store_true", help="only the selected workload")
    ap.add_argument("--no-full-parity", action="store_true",
                    help="skip the full-length oracle comparisons (and the host oracle run of C3)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries from the rocprofv3 passes in DIR (no GPU needed)")
    ap.add_argument("--profile-command", default="--steps 32 --warmup 0 --no-cpu-baseline --solves 0 --kernel-reps 4 "
                    "--kernel-phase-ms 0 --serving-requests 0 --no-time-to-error --no-full-parity --copy-probe",
                    help="the bench.py arguments the counter runs used (recorded in the summaries)")
    ap.add_argument("--stats-command", default="--gpus 1 --steps 20 --warmup 5 --no-cpu-baseline --solves 0 "
                    "--serving-requests 0 --no-time-to-error --no-full-parity",
                    help="the bench.py arguments the --kernel-trace --stats run used (the benchmark's timing)")
    args = ap.parse_args()

    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, os.path.join(ROOT, "profiles"), args.profile_command,
                           args.stats_command, args.kernel_reps)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1808_04960_amd as gw  # noqa: F401

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "serving":
        s = run_serving(args.serving_requests or 200, 2 << 30, 64, 8)
        print(json.dumps({"metric": METRIC, "value": s["cell_updates_per_s"], "unit": "cell-updates/s", "n_gpus": 1,
                          "steps": s["ticks"], "warmup": 0, "ms_per_step": None, "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": SERVING_DESC}, "serving": s, "roofline": None,
                          "cpu_baseline": None}), flush=True)
        return

    entries = profile_entries()
    sha = kernel_source_hash()
    W = WORKLOADS[args.workload]
    grid, U0 = W["make"]()
    R = W["R"]
    ncell = grid.ncells
    if "max_steps" in W and args.warmup + args.steps > W["max_steps"]:
        args.warmup = min(args.warmup, W["max_steps"] // 10)
        args.steps = W["max_steps"] - args.warmup
        log(f"timed run held to {args.warmup} + {args.steps} steps, inside the workload's span")

    solvers, timing, kern = time_workload(args.workload, W, grid, U0, args.steps, args.warmup, args.kernel_reps,
                                          args.kernel_phase_ms * 1e-3)

    if args.copy_probe:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {nbytes} bytes read + {nbytes} bytes written per launch")
        del a, b

    roof = roofline_of(W, grid, timing, kern, args.steps, "fp32", entries, sha)
    roof["fp64"] = roofline_of(W, grid, timing, kern, args.steps, "fp64", entries, sha)
    roof["fp64"].pop("fp64", None)

    # latency: full solves of the fp32 path
    lat = []
    acc = {}
    if W["t_final"] is not None and args.solves > 0:
        s = solvers["fp32"]
        for _ in range(args.solves):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.set_state(U0)
            s.run(W["t_final"])
            s.get_state()
            lat.append(time.perf_counter() - t0)
    if not args.no_full_parity:
        acc[args.workload] = full_length_accuracy(args.workload, W, grid, U0, solvers, True)
    for s in solvers.values():
        s.close()
    del solvers
    torch.cuda.empty_cache()

    # the other benchmark-scale workloads: timing, roofline, full-length parity
    workloads = {}
    if args.workload == "vortex2d" and not args.no_extra_workloads:
        for name in ("kh2d", "wave3d"):
            Wx = WORKLOADS[name]
            gx, Ux = Wx["make"]()
            sx, tx, kx = time_workload(name, Wx, gx, Ux, args.steps, args.warmup, args.kernel_reps,
                                       args.kernel_phase_ms * 1e-3)
            rx = roofline_of(Wx, gx, tx, kx, args.steps, "fp32", entries, sha)
            rx["fp64"] = roofline_of(Wx, gx, tx, kx, args.steps, "fp64", entries, sha)
            rx["fp64"].pop("fp64", None)
            workloads[name] = {
                "config": {"workload": Wx["desc"], "grid": list(gx.n[: gx.ndim]), "R": Wx["R"]},
                "value": gx.ncells * 3 * args.steps / tx["fp32"], "ms_per_step": tx["fp32"] / args.steps * 1e3,
                "fp64": {"value": gx.ncells * 3 * args.steps / tx["fp64"],
                         "ms_per_step": tx["fp64"] / args.steps * 1e3},
                "roofline": rx}
            if not args.no_full_parity and name == "wave3d":
                acc[name] = full_length_accuracy(name, Wx, gx, Ux, sx, False)
            for s in sx.values():
                s.close()
            del sx
            torch.cuda.empty_cache()
        if not args.no_full_parity:
            Wv = WORKLOADS["vortex3d"]
            gv, Uv = Wv["make"]()
            import paper_1808_04960_amd as gwm
            sv = {p: gwm.Solver(gv, 2, 12 * gv.dx[0], 3 * gv.dx[0], precision=p, U0=Uv) for p in ("fp32", "fp64")}
            acc["vortex3d"] = full_length_accuracy("vortex3d", Wv, gv, Uv, sv, False)
            for s in sv.values():
                s.close()
            del sv
            torch.cuda.empty_cache()

    # CPU oracle: bounded sample of the headline workload
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        dx = grid.dx[0]
        o = oracle.OracleSolver(grid, R, 12 * dx, 3 * dx, cfl=W.get("cfl", 0.4))
        Uo = U0.copy()
        t0 = time.perf_counter()
        steps = 0
        t_o = 0.0
        while True:
            t_o, n1 = o.run(Uo, 1e9, max_steps=1, t0=t_o)
            steps += n1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or el * (steps + 1) / steps > 30.0:
                break
        cpu = {"value": ncell * 3 * steps / el, "unit": "cell-updates/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"first {steps} SSP-RK3 steps of the same workload from t=0 ({el:.1f} s, float64)"}
        log(f"oracle: {steps} steps in {el:.1f} s on {oracle.threads()} threads")

    serving = None
    if args.workload == "vortex2d" and args.serving_requests > 0:
        serving = {"unconstrained": run_serving(args.serving_requests, 2 << 30, 64, 8),
                   "admission_binds": run_serving(args.serving_requests, 256 << 20, 64, 8, rate=200.0),
                   "workload": SERVING_DESC}

    tte = None
    if args.workload == "vortex2d" and not args.no_time_to_error:
        tte = time_to_error(5e-3)

    # the C3 oracle (a few minutes on the host) last, after every GPU timing
    if args.workload == "vortex2d" and not args.no_extra_workloads and not args.no_full_parity:
        Wk = WORKLOADS["kh2d"]
        gk, Uk = Wk["make"]()
        import paper_1808_04960_amd as gwm
        sk = {p: gwm.Solver(gk, 3, 12 * gk.dx[0], 3 * gk.dx[0], precision=p, U0=Uk) for p in ("fp32", "fp64")}
        acc["kh2d"] = full_length_accuracy("kh2d", Wk, gk, Uk, sk, True)
        for s in sk.values():
            s.close()

    cu32 = ncell * 3 * args.steps / timing["fp32"]
    cu64 = ncell * 3 * args.steps / timing["fp64"]
    out = {
        "metric": METRIC,
        "value": cu32,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": timing["fp32"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": W["desc"], "grid": list(grid.n[: grid.ndim]), "R": R,
                   "arithmetic": "float32 sweep, float64 state/dt/RK/sums"},
        "fp64": {"value": cu64, "ms_per_step": timing["fp64"] / args.steps * 1e3, "dtype": "f64"},
        "accuracy": acc,
        "latency": ({"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                     "solves": len(lat), "what": "upload + run to t_final + download, fp32 path"} if lat else None),
        "workloads": workloads,
        "serving": serving,
        "time_to_error": tte,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
