"""Host check (CPU only) of the single-pulse search's integer screen threshold: for each
(row, block, width) the search compares window sums against the smallest sum whose float64
S/N, evaluated as in the exact path, reaches the threshold (min_passing_sum). The harness
checks over 2 million random rows and widths that the returned sum reaches the threshold
and that the sum one below does not (so the screen passes exactly the cells whose best S/N
reaches the threshold), and the r = 0 and out-of-range cases. Compiled with hipcc as host
code."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_screen_threshold_is_the_exact_boundary(tmp_path):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "screen_check")
    cmd = [HIPCC, "-O2", "-std=c++17", "-ffp-contract=off", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "screen_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout + r.stderr
