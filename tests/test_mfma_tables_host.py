"""Host-logic test of the matrix-core dedispersion tables (CPU only). A scalar model of
the kernel's steps runs over the tables of a host-only plan and must reproduce the
brute-force sum D[d][t] = sum_c X[c][t + s[d][c]] exactly, for every time-tile, staging-depth
and channels-per-step configuration of the matrix-core variants (4 channels x 8 residuals
and 8 x 4 per step, and the two mixed by trial range), on shapes that span padded
channels, single-trial DM blocks, wide DM steps and 4096-channel blocks at the
63- and 31-tile channel-block limits. The harness is compiled with hipcc as host code."""

import os
import re
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
    exe = str(tmp_path_factory.mktemp("mfma") / "mfma_tables_check")
    cmd = [HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "mfma_tables_check.cpp"),
           os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "tiling.cpp"), os.path.join(CSRC, "tune.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


# cps 0 mixes the step shapes by trial range: split -1 takes the cost estimate's split,
# the others force it at that fraction of the trials (0: all 4-channel, 1: all 8-channel)
@pytest.mark.parametrize("tile,depth,max_tiles,cps,split", [
    (1024, 3, 63, 4, -1), (896, 5, 63, 4, -1), (768, 7, 63, 4, -1), (512, 3, 31, 4, -1), (480, 4, 31, 4, -1),
    (864, 3, 63, 8, -1), (512, 3, 31, 8, -1),
    (864, 3, 63, 0, -1), (864, 3, 63, 0, 0.5), (864, 3, 63, 0, 0.0), (864, 3, 63, 0, 1.0)])
def test_mfma_tables_reproduce_brute_force(harness, tile, depth, max_tiles, cps, split):
    r = subprocess.run([harness, str(tile), str(depth), str(max_tiles), str(cps), str(split)], capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout + r.stderr
    if cps == 0 and (split < 0 or 0 < split < 1):
        # the mixed tables must really mix: some case holds blocks of both shapes
        mixed = [(int(m.group(1)), int(m.group(2)))
                 for m in re.finditer(r"blocks (\d+) \((\d+) of 8 channels per step\)", r.stdout)]
        assert any(0 < n8 < n for n, n8 in mixed), r.stdout
