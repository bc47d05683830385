"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the binary128 table builder of the library (gp_tables.cpp) and the CPU oracle
are compiled with -fsanitize=address,undefined by gcc/g++ (no device code is
involved) and run over every scheme, R = 1..3, ell/dx from 6 to 192, and the
oracle's right-hand side and steps in 1D-3D with every boundary kind and both
flux corrections. Any out-of-bounds access, use after free, leak or undefined
behaviour aborts the driver and fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1808_04960_amd", "csrc")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
           OMP_NUM_THREADS="2")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++")


def _build_and_run(cmd, exe):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_table_builder_is_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tables")
    out = _build_and_run(["g++", "-std=c++17", *SAN, f"-I{CSRC}", os.path.join(HERE, "sanitize", "tables_driver.cpp"),
                          os.path.join(CSRC, "gp_tables.cpp"), "-lquadmath", "-o", exe], exe)
    assert "non-finite 0" in out


def test_oracle_is_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle")
    out = _build_and_run(["gcc", "-std=c11", *SAN, "-fopenmp", os.path.join(HERE, "sanitize", "oracle_driver.c"),
                          "-lm", "-o", exe], exe)
    assert "runs 54 non-finite 0" in out
