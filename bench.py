#!/usr/bin/env python3
"""Benchmark of the GP-WENO FD-Prim hot path on one MI355X.

A step is one SSP-RK3 step (CFL time step, three stages, each stage one fused
sweep per direction) of the whole grid. Default workload: the 2D isentropic
vortex, 512 x 512 periodic cells on [-5,5]^2, vortex strength 5, gamma = 1.4,
GP-R2 with ell = 12 dx, sigma = 3 dx, CFL 0.4, one period t = 10.

Reported (one JSON line):
  value       cell-updates/s per RK stage of the float32-sweep path (float64 state)
  fp64        the same for the all-float64 path
  accuracy    relative L1 of both paths against the float64 CPU oracle after the
              oracle's sample steps, and density L1 against the exact solution
              after full solves to t = 10
  latency     p50/p99 time-to-solution of full solves (upload, run to t = 10, download)
  serving     the continuous-batching request loop on a Poisson stream of problems
  time_to_error the paper's time-to-error comparison of GP-R1/R2/R3 with WENO-JS
  roofline    the dominant sweep kernel, timed with HIP events on its stream
  cpu_baseline the CPU oracle timed on a bounded sample of the same workload
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
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}  # MI355X published vector peaks
CSRC = os.path.join(ROOT, "paper_1808_04960_amd", "csrc")


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


def flops_per_cell_sweep(ndim: int, R: int, fp64: bool = False) -> int:
    """Algorithmic flops of one cell in one direction's sweep (FMA = 2, divide and
    square root = 1), counted from the per-cell formulas in the forms the sweep
    evaluates:
      cons->prim 3*ndim+3, eigen quantities 8, projection 6n (n = 2R+1),
      GP-WENO per field: indicators (R+1) * b_R, where b_R is one sub-stencil's
        sum of squared rows on mirrored sums and differences (b_1 = 10 for the
        plain 2x2 form, b_2 = 15, b_3 = 24), interpolation 2(R+1)(2R+1)
        (candidates pre-multiplied by their linear weights), weights and the two
        normalised sums: float32, ratios (e_min/e_m)^2, 11(R+1) + 2; float64,
        over a common denominator, (R+1) squares + p_R products (p = 0 / 3 / 6)
        + 8R + 8,
      back-projection 14, HLLC 43 + 5(ndim-1) + 3 nv (the flux and conserved
        vector of the one side the face takes),
      flux correction gathered by neighbour distance and difference 9 nv."""
    nv = 2 + ndim
    n = 2 * R + 1
    beta_window = {1: 10, 2: 15, 3: 24}[R]
    weights = (R + 1) + {1: 0, 2: 3, 3: 6}[R] + 8 * R + 8 if fp64 else 11 * (R + 1) + 2
    weno = (R + 1) * beta_window + 2 * (R + 1) * (2 * R + 1) + weights
    hllc = 43 + 5 * (ndim - 1) + 3 * nv
    return (3 * ndim + 3) + 8 + 6 * n + nv * weno + 14 + hllc + 9 * nv


WORKLOADS = {
    "vortex2d": dict(desc="2D isentropic vortex, 512x512 periodic on [-5,5]^2, strength 5, gamma 1.4, "
                          "GP-R2 (ell=12dx, sigma=3dx), SSP-RK3 CFL 0.4, t=10",
                     make=lambda: inputs.isentropic_vortex_2d(512), R=2, t_final=10.0, tag="vortex2d_512_R2"),
    "sine1d": dict(desc="1D sine density wave, N=128 periodic on [0,1], GP-R2, CFL 0.4, t=1",
                   make=lambda: inputs.sine_wave_1d(128), R=2, t_final=1.0, tag="sine1d_128_R2"),
    "kh2d": dict(desc="2D Kelvin-Helmholtz, 2048x1024 periodic on [0,2]x[0,1], GP-R3, CFL 0.4",
                 make=lambda: inputs.kelvin_helmholtz_2d(2048, 1024), R=3, t_final=None, tag="kh2d_2048x1024_R3"),
    "wave3d": dict(desc="3D density wave, 256^3 periodic on [0,1]^3, GP-R2, CFL 0.4",
                   make=lambda: inputs.density_wave_3d(256), R=2, t_final=None, tag="wave3d_256_R2"),
    "vortex3d": dict(desc="3D isentropic vortex (w=0), 256^3 periodic on [-5,5]^3, GP-R2, CFL 0.4",
                     make=lambda: inputs.isentropic_vortex_3d(256), R=2, t_final=None, tag="vortex3d_256_R2"),
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
                "Riemann data, FIFO admission by HBM footprint (budget 2 GiB, 64 slots), fp32 sweep arithmetic")


def run_serving(count, budget, slots, steps_per_tick, log):
    """Replays the serving stream through the continuous-batching server."""
    from paper_1808_04960_amd.serve import GpuExecutor, Server

    reqs = inputs.serving_stream(count=count, rate=20.0, seed=0)
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
    s["arrival_span_s"] = reqs[-1].arrival - reqs[0].arrival
    s["what"] = "latency = arrival to result on the host; cell_updates_per_s = work / (last completion - first arrival)"
    for j in rep.jobs:
        j.result = None
    ex.close()
    log(f"serving: {s['completed']}/{s['requests']} done, p50 {s['p50_ms']:.1f} ms, p99 {s['p99_ms']:.1f} ms, "
        f"{s['cell_updates_per_s']:.3e} cell-updates/s over {s['makespan_s']:.2f} s, peak {s['peak_active']} active")
    return s


TTE_DESC = ("2D isentropic vortex on [0,20]^2 (strength 5, background rho = u = v = p = 1, gamma 1.4), one "
            "period t = 20, ell = 1.2, sigma = 3 dx, CFL 0.4 without time-step reduction, SSP-RK3, float64 sweeps; "
            "L1 = 100 x mean |rho - rho(t=0)|")
TTE_CASES = (("weno-js", 2, (64, 96, 128, 192)), ("gp-weno", 1, (192, 256, 384, 512)),
             ("gp-weno", 2, (48, 64, 96, 128)), ("gp-weno", 3, (48, 64, 96, 128)))


def _interp_time(points, target):
    """Time at which the L1 error reaches target, interpolated log-log between the
    two grids that bracket it; None if no pair does."""
    pts = sorted(points, key=lambda p: -p[0])
    for (e0, t0), (e1, t1) in zip(pts, pts[1:]):
        if e0 >= target >= e1 and e0 > e1:
            f = math.log(e0 / target) / math.log(e0 / e1)
            return t0 * (t1 / t0) ** f
    return None


def time_to_error(target, log, cells_per_batch=1 << 20, max_copies=64):
    """The shape of the paper's time-to-error study (Sec. 6.2, Fig. (vortex_timing),
    Table (performace-time-to-error)) on the GPU. For each scheme and grid:
      single  -- wall time of one solve to t = 20 (state resident, graph replays);
      batched -- wall time per problem when copies of the problem fill the GPU
                 through the batched path (about cells_per_batch cells in flight);
    each interpolated log-log to the target L1 error and divided by WENO-JS's."""
    import torch

    import paper_1808_04960_amd as gw

    out = {"workload": TTE_DESC, "target_l1": target, "schemes": {}}
    for scheme, R, sizes in TTE_CASES:
        name = "WENO-JS" if scheme == "weno-js" else f"GP-R{R}"
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
    ref = out["schemes"]["WENO-JS"]
    for v in out["schemes"].values():
        for k in ("single_s", "batched_s", "cell_updates"):
            v[f"{k}_rel_weno_js"] = v[k] / ref[k] if v[k] and ref[k] else None
    out["paper_relative_time"] = {"GP-R1": 35.81, "GP-R2": 0.43, "GP-R3": 0.22, "WENO-JS": 1.0,
                                  "what": "CPU time on 4 cores with RK4, ell = 1.2 (the paper's table)"}
    return out


def traffic_from_profiles(kernel_name, tag):
    """HBM bytes per launch (fetched + written) of the kernel on the workload, from
    the committed rocprofv3 counter summary; None if there is none or the kernel
    source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    sha = kernel_source_hash()
    entries = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if len(parts) >= 5:
                entries[(parts[0], parts[1], parts[4])] = float(parts[2]) + float(parts[3])
    return entries.get((kernel_name.replace(" ", ""), sha, tag))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="vortex2d", choices=sorted(WORKLOADS) + ["serving"])
    ap.add_argument("--solves", type=int, default=5, help="full solves for latency and exact-solution error")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="oracle sample budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=100, help="back-to-back launches per timed kernel")
    ap.add_argument("--serving-requests", type=int, default=200, help="requests of the serving stream (0: skip)")
    ap.add_argument("--no-time-to-error", action="store_true", help="skip the time-to-error study")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1808_04960_amd as gw

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    W = WORKLOADS[args.workload]
    if args.workload == "serving":
        W = dict(desc=SERVING_DESC)
        s = run_serving(args.serving_requests or 200, 2 << 30, 64, 8, lambda m: print(f"[bench] {m}", file=sys.stderr))
        print(json.dumps({"metric": METRIC, "value": s["cell_updates_per_s"], "unit": "cell-updates/s", "n_gpus": 1,
                          "steps": s["ticks"], "warmup": 0, "ms_per_step": None, "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": SERVING_DESC}, "serving": s, "roofline": None,
                          "cpu_baseline": None}), flush=True)
        return
    grid, U0 = W["make"]()
    R = W["R"]
    dx = grid.dx[0]
    ncell = grid.ncells
    t_final = W["t_final"]
    t_run = 1e9  # timing runs never reach their end time

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if "max_steps" in W and args.warmup + args.steps > W["max_steps"]:
        args.warmup = min(args.warmup, W["max_steps"] // 10)
        args.steps = W["max_steps"] - args.warmup
        log(f"timed run held to {args.warmup} + {args.steps} steps, inside the workload's span")

    solvers = {}
    timing = {}
    for prec in ("fp32", "fp64"):
        s = gw.Solver(grid, R, 12 * dx, 3 * dx, precision=prec, cfl=W.get("cfl", 0.4), U0=U0)
        solvers[prec] = s
        s.run(t_run, max_steps=args.warmup)
        s.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n, _ = s.run(t_run, max_steps=args.steps)
        s.synchronize()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert n == args.steps
        timing[prec] = el
        log(f"{prec}: {args.steps} steps in {el * 1e3:.2f} ms -> {ncell * 3 * args.steps / el:.4e} cell-updates/s")

    # per-kernel launch durations: each launch of the step sequence
    # (gpweno_step_kernel k) repeated back to back between two HIP events on
    # the solver's stream. Every launch reads and writes the same buffers as in
    # a step, so a repeat does the same work; the host enqueues while the stream
    # is held in a bounded spin, so the kernels run back to back.
    nk = 3 * grid.ndim
    kern = {}
    for prec in ("fp32", "fp64"):
        s = solvers[prec]
        real = "float" if prec == "fp32" else "double"
        per_sym = {}
        for k in range(nk):
            s.set_state(U0)
            s.step(t_run)  # sets the end time and lifts the step limit
            s.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(s.stream):
                torch.cuda._sleep(int(2.4e9 * 0.01))
            e0.record(s.stream)
            for _ in range(args.kernel_reps):
                s.step_kernel(k)
            e1.record(s.stream)
            e1.synchronize()
            # sweeps of a stage run z, y, x; the x sweep finishes the stage
            d = grid.ndim - 1 - k % grid.ndim
            fin = d == 0
            # template arguments: ndim, dir, R, real type, finishes the stage,
            # indicator kind (0: GP), general boundaries (periodic: false)
            bcg = "true" if W.get("bcg", False) else "false"
            sym = f"sweep_kernel<{grid.ndim}, {d}, {R}, {real}, {'true' if fin else 'false'}, 0, {bcg}>"
            tk = e0.elapsed_time(e1) / args.kernel_reps * 1e-3
            per_sym.setdefault(sym, []).append(tk)
            log(f"  launch {k} (stage {k // grid.ndim + 1}, dir {d}): {tk * 1e6:.1f} us")
        for sym, ts in per_sym.items():
            kern[(prec, sym)] = (float(np.mean(ts)), len(ts))
            log(f"{sym}: {np.mean(ts) * 1e6:.1f} us per launch, {len(ts)} per step")

    if args.copy_probe:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {nbytes} bytes read + {nbytes} bytes written per launch")

    # accuracy and latency: full solves
    acc = {}
    lat = []
    if t_final is not None and args.solves > 0:
        rho_exact = U0[0]
        for prec in ("fp32", "fp64"):
            s = solvers[prec]
            reps = args.solves if prec == "fp32" else 1
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.set_state(U0)
                n, t = s.run(t_final)
                Ug = s.get_state()
                el = time.perf_counter() - t0
                if prec == "fp32":
                    lat.append(el)
            acc[f"{prec}_steps_to_t_final"] = int(n)
            if W.get("exact", True):  # the exact solution is the translated initial data
                acc[f"{prec}_density_l1_vs_exact"] = float(np.mean(np.abs(Ug[0] - rho_exact)))
                log(f"{prec}: solve to t={t:.3f} in {n} steps, density L1 vs exact "
                    f"{acc[f'{prec}_density_l1_vs_exact']:.3e}")
            else:
                log(f"{prec}: solve to t={t:.3f} in {n} steps")

    # CPU oracle: bounded sample of the same workload, then parity of both GPU paths
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        o = oracle.OracleSolver(grid, R, 12 * dx, 3 * dx, cfl=W.get("cfl", 0.4))
        Uo = U0.copy()
        t0 = time.perf_counter()
        steps = 0
        t_o = 0.0
        while True:
            t_o, n1 = o.run(Uo, t_run, max_steps=1, t0=t_o)
            steps += n1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or el * (steps + 1) / steps > 30.0:
                break
        cpu = {"value": ncell * 3 * steps / el, "unit": "cell-updates/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"first {steps} SSP-RK3 steps of the same workload from t=0 ({el:.1f} s, float64)"}
        log(f"oracle: {steps} steps in {el:.1f} s on {oracle.threads()} threads")
        for prec in ("fp32", "fp64"):
            s = solvers[prec]
            s.set_state(U0)
            s.run(t_run, max_steps=steps)
            Ug = s.get_state()
            acc[f"{prec}_rel_l1_vs_oracle"] = float(np.abs(Ug - Uo).sum() / np.abs(Uo).sum())
        acc["oracle_steps_compared"] = steps

    serving = None
    if args.workload == "vortex2d" and args.serving_requests > 0:
        serving = run_serving(args.serving_requests, 2 << 30, 64, 8, log)
        serving["workload"] = SERVING_DESC

    tte = None
    if args.workload == "vortex2d" and not args.no_time_to_error:
        tte = time_to_error(5e-3, log)

    cu32 = ncell * 3 * args.steps / timing["fp32"]
    cu64 = ncell * 3 * args.steps / timing["fp64"]
    def dominant(prec):
        syms = [k[1] for k in kern if k[0] == prec]
        return max(syms, key=lambda sym: kern[(prec, sym)][0] * kern[(prec, sym)][1])

    fl = flops_per_cell_sweep(grid.ndim, R) * ncell
    fl64 = flops_per_cell_sweep(grid.ndim, R, fp64=True) * ncell
    sym32, sym64 = dominant("fp32"), dominant("fp64")
    t32, t64 = kern[("fp32", sym32)][0], kern[("fp64", sym64)][0]
    achieved = fl / t32 / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS["fp32"], "traffic": traffic_from_profiles(sym32, W["tag"]), "kernel": sym32,
            "avg_launch_us": t32 * 1e6, "flops_per_launch": fl,
            "kernels_us": {k[1]: v[0] * 1e6 for k, v in kern.items()},
            "fp64": {"kernel": sym64, "avg_launch_us": t64 * 1e6, "achieved": fl64 / t64 / 1e12,
                     "flops_per_launch": fl64,
                     "peak": PEAK_TFLOPS["fp64"], "frac": fl64 / t64 / 1e12 / PEAK_TFLOPS["fp64"],
                     "traffic": traffic_from_profiles(sym64, W["tag"])}}
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
        "serving": serving,
        "time_to_error": tte,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
