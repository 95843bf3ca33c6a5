"""GPU parity of the decimated boxcar hierarchy (plan option boxcar_full_width): the
best-S/N plane bit for bit and the candidate lists exactly against the oracle, with the
float64 path and the integer-screened path, whole-signal and streamed in chunks."""

import numpy as np
import pytest

import oracle
from tests.gpu_util import assert_candidates_equal, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("w0,block", [(4, 32768), (1, 4096), (8, 8192)])
def test_hierarchy_matches_oracle(tiny, w0, block):
    from paper_2101_00941_amd import Plan
    w, x = tiny
    want = oracle.run(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"], block,
                      want_best=True, boxcar_full_width=w0)
    plan = Plan(w["nchan"], w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"], block,
                boxcar_full_width=w0)
    got = run_gpu(plan, x, w["nsamp"], cap=1 << 16)
    say(f"hierarchy w0 {w0} block {block}: {len(got['candidates'])} candidates")
    assert np.array_equal(got["best"], want["best"])
    assert_candidates_equal(got["candidates"], want["candidates"])
    got2 = run_gpu(plan, x, w["nsamp"], cap=1 << 16, want_best=False)
    assert_candidates_equal(got2["candidates"], want["candidates"])
    assert len(want["candidates"]) > 0


def test_hierarchy_streamed_equals_whole(tiny):
    import torch
    from paper_2101_00941_amd import Pipeline, Plan
    w, x = tiny
    want = oracle.run(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"], 4096,
                      boxcar_full_width=2)["candidates"]
    plan = Plan(w["nchan"], w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"], 4096,
                boxcar_full_width=2)
    host = torch.from_numpy(np.ascontiguousarray(x)).pin_memory()
    pipe = Pipeline(nstreams=2, max_beams=1, max_chunk=7000, hbm_budget=1 << 30, min_piece_work=-1)
    b = pipe.add_beam(plan)
    n, k = w["nsamp"], 0
    for a in range(0, n, 7000):
        m = min(7000, n - a)
        pipe.submit(b, host[:, a:a + m], nsamp=m, pitch=host.stride(0), tag=k, last=(a + m == n))
        k += 1
    got = []
    for _ in range(k):
        r = pipe.poll(timeout_us=20_000_000)
        assert r is not None and r["status"] == 0
        got.extend((int(c["dm_idx"]), int(c["t"]), int(c["width"]), float(c["snr"])) for c in r["cand"])
    pipe.close()
    got.sort(key=lambda c: (c[0], c[1]))
    assert_candidates_equal(got, want)
