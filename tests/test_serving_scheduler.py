"""Continuous-batching scheduler logic, on the modelled executor (no GPU):
admission by HBM footprint and slots, first-in first-out order, replay of the
Poisson arrival stream, retirement, and the latency statistics."""
import dataclasses

import numpy as np
import pytest

import inputs
from paper_1808_04960_amd.serve import PendingResult, Server, SimExecutor, footprint_bytes


@dataclasses.dataclass
class _Req:
    rid: int
    arrival: float
    n: int
    steps: int
    R: int = 2
    kind: str = "vortex"

    @property
    def grid(self):
        return inputs.grid2d(self.n, self.n)

    @property
    def cells(self):
        return self.n * self.n


class _Recorder(SimExecutor):
    """Tracks resident bytes and slot use at every tick."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.max_used = 0
        self.max_active = 0

    def set_active(self, handles):
        super().set_active(handles)   # raises for a set the executor refuses
        self.ever_active = getattr(self, "ever_active", set()) | {h.req.rid for h in self.active}

    def advance(self, k):
        used = sum(footprint_bytes(h.req.grid) for h in self.active)
        self.max_used = max(self.max_used, used)
        self.max_active = max(self.max_active, len(self.active))
        super().advance(k)


def test_footprint_matches_library_layout():
    g = inputs.grid2d(512, 512)
    one = 8 * 4 * 512 * 512
    assert footprint_bytes(g) == 4 * one + 8 * 4 * 1024
    g3 = inputs.grid3d(16, 16, 16)
    assert footprint_bytes(g3) == 4 * (8 * 5 * 4096) + 8 * 5 * 1024
    g1 = inputs.grid1d(100)
    assert footprint_bytes(g1) == 3 * (-(-8 * 3 * 100 // 256) * 256) + 8 * 3 * 1024


def test_poisson_stream_statistics():
    reqs = inputs.serving_stream(count=2000, rate=20.0, seed=0)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / 20.0) < 0.1 / 20.0
    assert set(r.n for r in reqs) == {64, 128, 256, 512, 1024}
    assert set(r.R for r in reqs) == {1, 2, 3}
    assert min(r.steps for r in reqs) >= 100 and max(r.steps for r in reqs) <= 500
    kinds = [r.kind for r in reqs]
    assert 0.45 < kinds.count("vortex") / len(kinds) < 0.55
    # reproducible from the seed
    again = inputs.serving_stream(count=20, rate=20.0, seed=0)
    assert [(r.arrival, r.n, r.R, r.steps, r.kind, r.seed) for r in again] == \
           [(r.arrival, r.n, r.R, r.steps, r.kind, r.seed) for r in reqs[:20]]


def test_everything_completes_within_budget_and_slots():
    reqs = inputs.serving_stream(count=200, rate=20.0, seed=1)
    budget = 2 << 30
    ex = _Recorder(rate=5e9)
    rep = Server(ex, hbm_budget=budget, max_slots=16, steps_per_tick=8).run(reqs)
    s = rep.summary()
    assert s["completed"] == 200 and s["failed"] == 0 and s["rejected"] == 0
    assert ex.max_used <= budget and rep.peak_bytes <= budget
    assert ex.max_active <= 16 and rep.peak_active <= 16
    for j in rep.jobs:
        assert j.admitted >= j.req.arrival - 1e-12      # never before it arrives
        assert j.finished >= j.admitted
        assert j.steps_done == j.req.steps
    # exact accounting of the work done
    total = sum(3.0 * r.steps * r.n * r.n for r in reqs)
    assert rep.cell_updates == pytest.approx(total)


def test_fifo_admission_order():
    reqs = inputs.serving_stream(count=100, rate=50.0, seed=2)
    ex = SimExecutor(rate=2e9)
    rep = Server(ex, hbm_budget=1 << 30, max_slots=8).run(reqs)
    assert ex.admitted == [r.rid for r in sorted(reqs, key=lambda r: r.arrival)]
    adm = [j.admitted for j in rep.jobs]
    assert adm == sorted(adm)


def test_head_of_line_blocking_and_backfill_of_freed_memory():
    """A large request waits for memory; smaller ones behind it wait too (FIFO);
    when the running job retires, both are admitted while nothing else runs."""
    big = _Req(0, 0.0, 512, 100)
    blocker = _Req(1, 0.0, 512, 50)
    small = _Req(2, 0.001, 64, 10)
    budget = footprint_bytes(big.grid) + footprint_bytes(small.grid) + 1
    ex = SimExecutor(rate=1e9)
    rep = Server(ex, hbm_budget=budget, max_slots=8, steps_per_tick=10).run([big, blocker, small])
    jb = {j.req.rid: j for j in rep.jobs}
    assert jb[0].admitted == 0.0
    assert jb[1].admitted >= jb[0].finished      # needed the memory of job 0
    assert jb[2].admitted >= jb[1].admitted      # FIFO behind job 1
    assert all(j.status == "done" for j in rep.jobs)


def test_oversized_request_is_rejected_and_failures_are_isolated():
    reqs = [_Req(0, 0.0, 1024, 20), _Req(1, 0.0, 64, 20), _Req(2, 0.0, 64, 20), _Req(3, 0.0, 64, 20)]
    budget = footprint_bytes(reqs[1].grid) * 3
    ex = SimExecutor(rate=1e9, fail_rids={2})
    rep = Server(ex, hbm_budget=budget, max_slots=8, steps_per_tick=4).run(reqs)
    st = {j.req.rid: j.status for j in rep.jobs}
    assert st == {0: "rejected", 1: "done", 2: "failed", 3: "done"}


def test_latency_percentiles():
    reqs = inputs.serving_stream(count=150, rate=30.0, seed=3)
    rep = Server(SimExecutor(rate=3e9), hbm_budget=4 << 30, max_slots=32).run(reqs)
    lat = np.array([j.finished - j.req.arrival for j in rep.jobs])
    s = rep.summary()
    assert s["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert s["p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_a_request_whose_admission_raises_fails_alone():
    """Admission raising (e.g. invalid parameters or an allocation failure) ends
    that request as failed, takes no memory, and the loop serves the rest."""
    reqs = [_Req(i, 0.001 * i, 64, 12) for i in range(6)]
    ex = _Recorder(rate=1e9, admit_raises={2})
    rep = Server(ex, hbm_budget=footprint_bytes(reqs[0].grid) * 2, max_slots=4, steps_per_tick=4).run(reqs)
    st = {j.req.rid: j.status for j in rep.jobs}
    assert st == {0: "done", 1: "done", 2: "failed", 3: "done", 4: "done", 5: "done"}
    assert "admission of request 2" in rep.jobs[2].error
    assert ex.max_used <= footprint_bytes(reqs[0].grid) * 2
    assert rep.summary()["failed"] == 1


def test_a_request_the_batch_refuses_fails_alone():
    """The batch refusing a set (e.g. the device-side tables of one member) is
    traced to the member it refuses alone: that request fails, its footprint is
    released, and the set is rebuilt from the others, which finish."""
    reqs = [_Req(i, 0.0, 64, 16) for i in range(5)]
    ex = _Recorder(rate=1e9, set_refuses={3})
    rep = Server(ex, hbm_budget=footprint_bytes(reqs[0].grid) * 5, max_slots=8, steps_per_tick=4).run(reqs)
    st = {j.req.rid: j.status for j in rep.jobs}
    assert st == {0: "done", 1: "done", 2: "done", 3: "failed", 4: "done"}
    assert rep.jobs[3].steps_done == 0 and "refused" in rep.jobs[3].error
    assert 3 not in ex.ever_active and {0, 1, 2, 4} <= ex.ever_active


class _SlowCopy(PendingResult):
    """A result that arrives after a fixed number of polls, with its bytes
    still held until then."""

    def __init__(self, ex, rid, polls):
        self.ex, self.rid, self.left = ex, rid, polls
        ex.held.add(rid)

    def done(self):
        self.left -= 1
        return self.left <= 0

    def value(self):
        return ("result", self.rid)

    def release(self):
        self.ex.held.discard(self.rid)


class _CopyingExecutor(_Recorder):
    """Retires with results still on their way (copied back while the next
    steps run), as the GPU executor does."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.held = set()
        self.max_bytes = 0

    def retire(self, handle, keep):
        return _SlowCopy(self, handle.req.rid, 3) if keep else None

    def advance(self, k):
        held = sum(footprint_bytes(_Req(r, 0.0, self.sizes[r], 1).grid) for r in self.held)
        used = sum(footprint_bytes(h.req.grid) for h in self.active)
        self.max_bytes = max(self.max_bytes, used + held)
        super().advance(k)


def test_results_still_on_their_way_hold_their_memory_until_they_land():
    """A job completes when its result has landed: its latency includes the
    copy, its footprint stays counted until then (resident plus still-held
    bytes never exceed the budget), and every result lands before run ends."""
    reqs = [_Req(i, 0.0005 * i, n, steps) for i, (n, steps) in
            enumerate([(128, 12), (96, 20), (128, 8), (64, 30), (96, 16), (128, 10)])]
    budget = 2 * footprint_bytes(inputs.grid2d(128, 128)) + 1
    ex = _CopyingExecutor(rate=2e9)
    ex.sizes = {r.rid: r.n for r in reqs}
    rep = Server(ex, hbm_budget=budget, max_slots=8, steps_per_tick=4).run(reqs, keep_results=True)
    assert all(j.status == "done" and j.result == ("result", j.req.rid) for j in rep.jobs)
    assert not ex.held
    assert ex.max_bytes <= budget
    for j in rep.jobs:
        assert j.finished > j.admitted
