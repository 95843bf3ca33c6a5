"""Host-logic test of the quad dedispersion tables (layout 7, CPU only). A scalar model
of the kernel's steps (chunked staging from aligned dwords, byte alignment and 4x4
transpose, per-trial dword sums at the recorded offsets) runs over the tables of a
host-only plan and must reproduce D[d][t] = sum_c X[c][t + s[d][c]] exactly. It also
checks that no dword load leaves its row on tiles the kernel runs without load guards,
and that every LDS access stays inside the step buffer. Shapes span padded channel
quads, single-channel plans, short blocks, steep and shallow DM steps on the 4096-channel
survey band. The harness is compiled with hipcc as host code."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2101_00941_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("quad") / "quad_tables_check")
    cmd = [HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "quad_tables_check.cpp"),
           os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "tiling.cpp"), os.path.join(CSRC, "tune.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


# (time tile, staging chunks per step) of the quad variants, plus a tight budget that
# forces short blocks
@pytest.mark.parametrize("tile,chunks", [(1024, 32), (512, 16), (1024, 8), (2048, 64)])
def test_quad_tables_reproduce_brute_force(harness, tile, chunks):
    r = subprocess.run([harness, str(tile), str(chunks)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout + r.stderr
