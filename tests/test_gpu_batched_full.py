"""Parity of the batched form at its full size: 64 beams of uneven shape (nchan 1024,
2048 or 4096; nsamp U[2^16, 2^20]; 500-3000 trials of the doubling-step plan; 0-5
injected pulses each; 85 GB of input generated on the device), run by aa_batch_run with
the autotuned variant as the batched bench does. Three beams (the smallest, a middle one
and the one with the most work) are copied to the host, and the oracle dedisperses every
500th trial and the trials around each of their pulses over the full time range and runs
its own search; the batched candidate lists restricted to those trials must equal it."""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from tests.gpu_util import assert_candidates_equal, say

pytestmark = pytest.mark.gpu


def _rows(b, ndm):
    dms = np.asarray(b["dms"])
    rows = set(range(0, ndm, 500))
    for p in b["pulses"]:
        r = int(np.argmin(np.abs(dms - p.dm)))
        rows |= {q for q in range(r - 2, r + 3) if 0 <= q < ndm}
    return sorted(rows)


def _runs(rows):
    out = []
    for r in rows:
        if out and r == out[-1][1] + 1:
            out[-1][1] = r
        else:
            out.append([r, r])
    return out


def test_batched_64_beams_sampled_against_oracle():
    import torch
    from paper_2101_00941_amd import Plan, batch_run, candidates_as_tuples
    from synth.filterbank_torch import make_filterbank_torch
    from synth.workloads import batched_beams
    bs = batched_beams(nbeams=64)
    beams = []
    for b in bs:
        x = make_filterbank_torch(b["nchan"], b["nsamp"], b["f_top"], b["foff"], b["tsamp"], b["pulses"],
                                  seed=b["seed"], device="cuda")
        plan = Plan(b["nchan"], b["nsamp"], b["f_top"], b["foff"], b["tsamp"], b["dms"], b["widths"], b["threshold"],
                    b["stat_block"])
        beams.append((plan, x, b["nsamp"]))
    torch.cuda.synchronize()
    say(f"batched: 64 beams, {sum(x.numel() for _, x, _ in beams) / 1e9:.1f} GB on the device")
    work = torch.empty(120 << 30, dtype=torch.uint8, device="cuda")
    cap = 1 << 20
    cands, counts, info = batch_run(beams, variant=-1, work=work, cap=cap)
    torch.cuda.synchronize()
    del work
    say(f"  batch: {info['groups']} launches, variant {info['variant']}")
    say(f"  candidates per beam: max {int(max(counts))}, total {int(sum(counts))}")
    assert info["groups"] >= 1 and all(c < cap for c in counts)
    work_units = [p.info["ndm"] * p.info["n_dd"] * p.info["nchan"] for p, _, _ in beams]
    order = np.argsort(work_units)
    picks = sorted({int(order[0]), int(order[len(order) // 2]), int(order[-1])})
    nthreads = max(1, min(16, os.cpu_count() or 1))
    for i in picks:
        b, (plan, x, n) = bs[i], beams[i]
        ndm, T, B, M = plan.info["ndm"], plan.info["n_start"], plan.info["stat_block"], plan.info["maxshift"]
        s = plan.shifts().astype(np.int64)
        assert np.array_equal(s, oracle.shift_table(b["dms"], b["nchan"], b["f_top"], b["foff"], b["tsamp"]))
        xh = x[:, :n].cpu().numpy()
        rows = _rows(b, ndm)
        need = sorted({q for r in rows for q in (r - 1, r, r + 1) if 0 <= q < ndm})
        with ThreadPoolExecutor(nthreads) as pool:
            D = dict(pool.map(lambda q: (q, oracle.dedisperse_rows(xh, s, [q], n, M)[0]), need))
        want = []
        for a, z in _runs(rows):
            lo, hi = max(a - 1, 0), min(z + 1, ndm - 1)
            c, _ = oracle.single_pulse(np.stack([D[q] for q in range(lo, hi + 1)]), 0, 0, T, T, b["widths"],
                                       b["threshold"], B, row0=lo, ndm=ndm, report_rows=list(range(a, z + 1)))
            want.extend(c)
        want.sort(key=lambda c: (c[0], c[1]))
        rs = set(rows)
        have = [c for c in candidates_as_tuples(cands[i]) if c[0] in rs]
        say(f"  beam {i}: {b['nchan']} ch x {n}, {ndm} trials, {len(rows)} checked trials, "
            f"{len(want)} oracle candidates, {len(have)} batched")
        assert counts[i] < cap
        assert_candidates_equal(have, want)
