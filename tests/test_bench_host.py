"""Host-side checks of the benchmark's bookkeeping (no GPU): the algorithmic
flop and byte counts the roofline divides by, the profile summarizer's split of
traced launches, the source hash that keys the counter tables, and the refusal
of more than one GPU."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_flops_per_cell_and_direction():
    """The per-cell tally of the path's steps: eigen quantities 10, projection 10n, per field
    4(R+1)^2 + 2(R+1)^2(R+2) + 13(R+1), back-projection 16, HLLC 90, correction
    and difference 9 nv."""
    assert bench.flops_per_cell_dir(2, 2) == 790
    assert bench.flops_per_cell_dir(2, 3) == 1326
    assert bench.flops_per_cell_dir(3, 2) == 946
    # a finishing sweep adds the stage combination, 4 nv per cell
    assert bench.flops_per_launch(2, 2, 512 * 512, True) == (790 + 16) * 512 * 512
    assert bench.flops_per_launch(3, 2, 256**3, False) == 946 * 256**3


def test_evaluated_form_counts():
    assert [bench.flops_per_cell_dir_evaluated(n, R) for n, R in ((2, 2), (3, 2), (2, 3))] == [597, 727, 961]
    assert [bench.flops_per_cell_dir_evaluated(n, R, True) for n, R in ((2, 2), (3, 2), (2, 3))] == [577, 702, 945]


def test_algorithmic_bytes_per_step():
    """(8/3) nv float64 values per cell-update, three stages per step: 5.37 GB
    for the 256^3 wave, 67.1 MB for the 512^2 vortex."""
    assert bench.algorithmic_bytes_per_step(3, 256**3) == pytest.approx(8 * 5 * 8 * 256**3)
    assert bench.algorithmic_bytes_per_step(2, 512 * 512) == pytest.approx(67108864.0)


def _trace(path, launches):
    """A rocprofv3-style kernel trace: (name, start, end) in ns."""
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for name, t0, t1 in launches:
            w.writerow(["KERNEL_DISPATCH", name, t0, t1])


def test_trace_split_separates_back_to_back_launches(tmp_path):
    y = "void gpw::sweep_kernel<2, 1, 2, float, false, 0, false, 2>(gpw::SweepArgs<float>)"
    x = "void gpw::sweep_kernel<2, 0, 2, float, true, 0, false, 2>(gpw::SweepArgs<float>)"
    launches, t = [], 0
    for _ in range(3):                      # replayed steps: y, x alternate (10 and 8 us)
        for name, d in ((y, 10_000), (x, 8_000)):
            launches.append((name, t, t + d))
            t += d + 500
    for name, d in ((y, 9_000), (x, 7_000)):   # four back-to-back launches of each
        for _ in range(4):
            launches.append((name, t, t + d))
            t += d + 100
    launches.append(("__amd_rocclr_copyBuffer", t, t + 50))
    path = tmp_path / "trace.csv"
    _trace(path, launches[::-1])            # rows need not be in time order
    s = bench._trace_split(str(path), 4)
    ky, kx = bench._short_name(y), bench._short_name(x)
    assert s[ky]["b2b"] == (4, 9.0) and s[ky]["seq"] == (3, 10.0)
    assert s[kx]["b2b"] == (4, 7.0) and s[kx]["seq"] == (3, 8.0)
    assert set(s) == {ky, kx}


def test_source_hash_ignores_comments_and_whitespace():
    code = "int f(int a) {\n  return a + 1;  // add one\n}\n/* block\n comment */"
    assert bench._code_only(code) == bench._code_only("int f(int a){ return a+1; }")
    assert bench._code_only(code) != bench._code_only("int f(int a){ return a+2; }")
    assert len(bench.kernel_source_hash()) == 16


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_committed_profiles_match_the_device_sources():
    """The counter tables the benchmark reads (profiles/traffic.txt,
    valu_busy.txt) were taken with the device sources as they are: a kernel
    change without a new profile fails here instead of silently reporting no
    traffic."""
    sha = bench.kernel_source_hash()
    for name in ("traffic.txt", "valu_busy.txt"):
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            rows = [line.split() for line in fh if line.strip() and not line.startswith("#")]
        assert rows and all(r[1] == sha for r in rows), name
    with open(os.path.join(ROOT, "profiles", "kernel_stats_vortex2d_512_R2.txt")) as fh:
        assert f"sha256[:16] = {sha}" in fh.read()


def test_committed_flop_ratios_are_per_lane():
    """SQ_INSTS_VALU_FLOPS_* and SQ_INSTS_VALU are both wave-level counts, so
    their ratio is the hardware flops per lane-instruction: between 0.5 and 2
    (an FMA counts 2) for every sweep, and so is the algorithmic ratio."""
    for tag in ("vortex2d_512_R2", "kh2d_2048x1024_R3", "wave3d_256_R2"):
        with open(os.path.join(ROOT, "profiles", f"counters_{tag}.txt")) as fh:
            vals = {}
            for line in fh:
                parts = line.split()
                if len(parts) == 2 and parts[0].endswith("flops_per_lane_instr"):
                    vals.setdefault(parts[0], []).append(float(parts[1]))
        assert set(vals) == {"hw_flops_per_lane_instr", "alg_flops_per_lane_instr"}, tag
        for v in vals.values():
            assert all(0.5 < x < 2.0 for x in v), (tag, v)


def test_limiter_reads_the_counters():
    """The 512^2 y sweep (VALU busy 0.50, 25 % of HBM) is latency-bound; the
    large-grid sweeps (0.78-0.93) are VALU-issue bound."""
    assert bench.limiter(0.50, 0.25).startswith("latency")
    assert bench.limiter(0.93, 0.51).startswith("VALU")
    assert bench.limiter(0.40, 0.70).startswith("HBM")
    assert bench.limiter(None, None) is None


def test_kernel_timing_phase_scales_short_passes_only():
    """A first pass shorter than the phase is followed by one scaled to fill
    it; a long enough pass (or a phase of 0) is used as it is."""
    assert bench.phase_reps(100, 0.0055, 0.2) == 3637   # 512^2 sweeps: 5.5 ms -> 0.2 s
    assert bench.phase_reps(100, 0.3, 0.2) is None
    assert bench.phase_reps(4, 0.001, 0.0) is None
    assert bench.phase_reps(100, 0.0, 0.2) == 100_000  # scaled by at most 1000
