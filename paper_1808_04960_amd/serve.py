"""Continuous batching of independent Euler problems on one GPU.

Requests arrive over time and are replayed against a clock. A request is admitted
when a slot is free and its HBM footprint (state plus stage workspace) fits the
budget. Admitted problems stay resident on the device. The scheduler advances all
of them together, a few steps per tick: each step is one batched launch per sweep
and per group of problems of one kind (dimension, R, precision, tables;
``gpweno_batch_run``, replayed from captured graphs, one per kind, the kinds
on streams of their own so that they run side by side).
A problem that reaches its step count is copied back and its memory released,
which lets the next waiting requests in while the others keep running.

The batch's step graphs are captured once per set of problem kinds: admitting or
retiring a problem rewrites the batch's device work tables with stream-ordered
copies, and a new problem's initial state is uploaded on a stream of its own,
so neither waits for the batches in flight. A finished problem's result is
copied back on a stream of its own too, while the next steps run; the request
completes (and its memory is released) once the copy has landed. The host waits
once per tick, for the progress poll.

Admission is first-in first-out: a request that does not fit blocks the ones
behind it (no starvation of large problems). A request larger than the whole
budget is rejected.

Failures stay with their request: one the device flags as non-physical, one
whose admission raises (e.g. invalid parameters, an allocation failure), and
one the batch refuses when the set changes, each end as "failed" with their
footprint released, while the others keep running.

Executors:
  ``GpuExecutor`` -- the device path (``Solver`` + ``Batch``);
  ``SimExecutor`` -- a modelled executor on a virtual clock, used to test the
                     scheduling logic without a GPU.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

PARTIAL_SUMS = 1024  # partial sums of the conservation reduction in the workspace


def footprint_bytes(grid) -> int:
    """Device bytes one problem holds: float64 state, two RK stage states, the
    direction accumulator (ndim > 1) and the reduction partials."""
    nv = 2 + grid.ndim
    one = -(-8 * nv * grid.ncells // 256) * 256
    arrays = 3 + (1 if grid.ndim > 1 else 0)
    return arrays * one + -(-8 * nv * PARTIAL_SUMS // 256) * 256


@dataclasses.dataclass
class Job:
    req: object
    footprint: int
    status: str = "waiting"  # waiting, active, done, failed, rejected
    admitted: float = float("nan")
    finished: float = float("nan")
    steps_done: int = 0
    handle: object = None
    result: object = None
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.req.arrival


class PendingResult:
    """A result still being copied to the host: ``done()`` polls, ``value()``
    waits for it and returns it, ``release()`` frees what it holds."""

    def done(self) -> bool:  # pragma: no cover - interface
        raise NotImplementedError

    def value(self):  # pragma: no cover - interface
        raise NotImplementedError

    def release(self):  # pragma: no cover - interface
        pass


@dataclasses.dataclass
class Report:
    jobs: list
    makespan: float
    cell_updates: float
    peak_bytes: int
    peak_active: int
    ticks: int

    def latencies(self):
        return np.array([j.latency for j in self.jobs if j.status == "done"])

    def summary(self):
        lat = self.latencies()
        done = [j for j in self.jobs if j.status == "done"]
        return {
            "requests": len(self.jobs),
            "completed": len(done),
            "failed": sum(j.status == "failed" for j in self.jobs),
            "rejected": sum(j.status == "rejected" for j in self.jobs),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
            "makespan_s": self.makespan,
            "cell_updates_per_s": self.cell_updates / self.makespan if self.makespan > 0 else None,
            "peak_resident_bytes": self.peak_bytes,
            "peak_active": self.peak_active,
            "ticks": self.ticks,
        }


class Server:
    def __init__(self, executor, hbm_budget: int, max_slots: int = 64, steps_per_tick: int = 8):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.k = int(steps_per_tick)

    def run(self, requests, keep_results=False):
        ex = self.ex
        jobs = [Job(r, ex.footprint(r)) for r in sorted(requests, key=lambda r: (r.arrival, r.rid))]
        pending = list(jobs)
        waiting = []
        active = []
        used = 0
        peak_bytes = 0
        peak_active = 0
        ticks = 0
        cell_updates = 0.0
        t0 = ex.now()
        first_arrival = jobs[0].req.arrival if jobs else 0.0
        finishing = []   # (job, PendingResult): done on the device, result on its way

        def land(block):
            """Completes the jobs whose results have arrived (all of them if
            block); returns the footprint released."""
            nonlocal finishing
            freed, rest = 0, []
            for j, r in finishing:
                if block or r.done():
                    j.result = r.value()
                    r.release()
                    j.finished = ex.now() - t0
                    freed += j.footprint
                else:
                    rest.append((j, r))
            finishing = rest
            return freed

        while pending or waiting or active or finishing:
            used -= land(False)
            now = ex.now() - t0
            while pending and pending[0].req.arrival <= now:
                j = pending.pop(0)
                if j.footprint > self.budget:
                    j.status = "rejected"
                    j.finished = now
                else:
                    waiting.append(j)
            changed = False
            while waiting and len(active) < self.max_slots and used + waiting[0].footprint <= self.budget:
                j = waiting.pop(0)
                try:
                    j.handle = ex.admit(j.req)
                except Exception as e:  # noqa: BLE001 - the request fails, the server goes on
                    j.status = "failed"
                    j.error = repr(e)
                    j.finished = ex.now() - t0
                    continue
                j.status = "active"
                j.admitted = ex.now() - t0
                used += j.footprint
                active.append(j)
                changed = True
            peak_bytes = max(peak_bytes, used)
            peak_active = max(peak_active, len(active))
            if changed:
                active, refused = self._set_active(active)
                for j in refused:
                    used -= self._fail(j, ex.now() - t0)
            if not active:
                if finishing:
                    used -= land(True)
                elif pending:
                    ex.idle_until(t0 + pending[0].req.arrival)
                continue
            ex.advance(self.k)
            ticks += 1
            nsteps, err = ex.progress()
            retired = []
            for j, n, e in zip(active, nsteps, err):
                cell_updates += (int(n) - j.steps_done) * 3.0 * j.req.cells
                j.steps_done = int(n)
                if e or n >= j.req.steps:
                    res = ex.retire(j.handle, keep_results and not e)
                    j.handle = None
                    j.status = "failed" if e else "done"
                    retired.append(j)
                    if isinstance(res, PendingResult):
                        finishing.append((j, res))
                    else:
                        j.result = res
                        j.finished = ex.now() - t0
                        used -= j.footprint
            if retired:
                active = [j for j in active if j.handle is not None]
                active, refused = self._set_active(active)
                for j in refused:
                    used -= self._fail(j, ex.now() - t0)
        makespan = max((j.finished for j in jobs), default=0.0) - first_arrival
        return Report(jobs, makespan, cell_updates, peak_bytes, peak_active, ticks)

    def _set_active(self, active):
        """Hands the active jobs to the executor. If it refuses the set, the jobs
        are added back one at a time: those it refuses alone are returned as
        refused, the rest form the new set (an executor that refuses even
        that raises)."""
        try:
            self.ex.set_active([j.handle for j in active])
            return active, []
        except Exception:  # noqa: BLE001 - find the job(s) it refuses
            pass
        ok, refused = [], []
        for j in active:
            try:
                self.ex.set_active([h.handle for h in ok] + [j.handle])
                ok.append(j)
            except Exception as e:  # noqa: BLE001
                j.error = repr(e)
                refused.append(j)
        self.ex.set_active([j.handle for j in ok])
        return ok, refused

    def _fail(self, j, now):
        """Ends an active job as failed; returns the footprint it released."""
        try:
            self.ex.retire(j.handle, False)
        except Exception:  # noqa: BLE001 - its resources go with the handle
            pass
        j.handle = None
        j.status = "failed"
        j.finished = now
        return j.footprint


class GpuExecutor:
    """Problems resident on the GPU, advanced by one ``Batch`` on one stream."""

    def __init__(self, precision="fp32", device=None):
        import torch

        from . import Batch

        self.torch = torch
        self.precision = precision
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = torch.cuda.Stream(self.device)
        self.upload = torch.cuda.Stream(self.device)
        self.copy = torch.cuda.Stream(self.device)
        self.batch = Batch(self.stream)

    def now(self):
        return time.perf_counter()

    def idle_until(self, t):
        dt = t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)

    def footprint(self, req):
        return footprint_bytes(req.grid)

    def admit(self, req):
        from . import Solver

        dx = req.grid.dx[0]
        s = Solver(req.grid, req.R, 12 * dx, 3 * dx, gamma=req.gamma, precision=self.precision,
                   positivity_fallback=(req.kind == "quadrant"), device=self.device.index, stream=self.stream)
        # the initial state goes up on a stream of its own; the serving stream
        # waits for it, the host does not wait for the batches in flight
        s.set_state(req.state(), upload_stream=self.upload)
        s.set_end(1e30, req.steps)
        return s

    def set_active(self, handles):
        self.batch.set(handles)

    def advance(self, k):
        self.batch.run(k)

    def progress(self):
        _, _, ns, err = self.batch.status()
        return ns, err

    def retire(self, handle, keep):
        """Called while the stream is idle (right after the progress poll). The
        context goes at once; with keep, the state is copied into pinned host
        memory on the copy stream, behind everything enqueued so far, and the
        returned PendingResult holds the device state until the copy is done."""
        torch = self.torch
        handle.close()
        handle.workspace = None
        if not keep:
            handle.state = None
            return None
        state = handle.state
        handle.state = None
        host = torch.empty(state.shape, dtype=state.dtype, pin_memory=True)
        self.copy.wait_stream(self.stream)
        with torch.cuda.stream(self.copy):
            host.copy_(state, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy)
        return _CopyBack(state, host, ev)

    def close(self):
        self.batch.close()


class _CopyBack(PendingResult):
    """A finished problem's state on its way to pinned host memory."""

    def __init__(self, state, host, event):
        self.state, self.host, self.event = state, host, event

    def done(self):
        return self.event.query()

    def value(self):
        self.event.synchronize()
        return self.host.numpy()

    def release(self):
        self.state = None


class SimExecutor:
    """Modelled executor: problems progress at a fixed aggregate rate of
    cell-updates per second on a virtual clock (scheduler tests, no GPU)."""

    @dataclasses.dataclass
    class Handle:
        req: object
        steps: int = 0

    def __init__(self, rate=5e9, fail_rids=(), admit_raises=(), set_refuses=()):
        """fail_rids: requests the device flags non-physical after their first
        step; admit_raises: requests whose admission raises; set_refuses:
        requests whose handle the batch refuses (set_active raises while it is
        in the set)."""
        self.t = 0.0
        self.rate = float(rate)
        self.active = []
        self.fail_rids = set(fail_rids)
        self.admit_raises = set(admit_raises)
        self.set_refuses = set(set_refuses)
        self.admitted = []

    def now(self):
        return self.t

    def idle_until(self, t):
        self.t = max(self.t, t)

    def footprint(self, req):
        return footprint_bytes(req.grid)

    def admit(self, req):
        if req.rid in self.admit_raises:
            raise RuntimeError(f"admission of request {req.rid} failed")
        self.admitted.append(req.rid)
        return SimExecutor.Handle(req)

    def set_active(self, handles):
        if any(h.req.rid in self.set_refuses for h in handles):
            raise RuntimeError("batch refused the set")
        self.active = list(handles)

    def advance(self, k):
        work = 0.0
        for h in self.active:
            take = min(k, h.req.steps - h.steps)
            work += take * 3.0 * h.req.cells
            h.steps += take
        self.t += work / self.rate

    def progress(self):
        ns = np.array([h.steps for h in self.active], dtype=np.int64)
        err = np.array([1 if (h.req.rid in self.fail_rids and h.steps > 0) else 0 for h in self.active])
        return ns, err

    def retire(self, handle, keep):
        return None
