"""Parity at the survey size: 4096 channels x 2^20 samples, 3000 DM trials (doubling
steps to DM 1998), boxcars 1..256, threshold 6, in the configuration the benchmark
times (resident input, one stream, autotuned dedispersion variant).

The whole plane (3000 x 1,012,255 int32, 12 GB) is beyond the oracle, so the
oracle checks sampled outputs, each computed on its own:
  * dedispersion: random (trial, sample) pairs, every trial at the first and last
    samples and at a random one, and full 32768-sample runs of a few trials, for
    the autotuned variant, every matrix-core and quad shift-and-add variant and one
    variant of each other kernel family;
  * candidates (plain and per-range decimated): every 100th trial and the two trials on each side of every
    injected pulse's DM (127 rows, chosen from the signal model), over the full
    time range. The oracle dedisperses each of those rows and its neighbours over
    all samples (220 rows, threaded over the host cores) and runs its own search.
    The GPU list restricted to those rows must equal the oracle's exactly.
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import assert_candidates_equal, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def survey():
    import torch
    from paper_2101_00941_amd import Plan
    from synth.workloads import make_input, workload
    w = workload("survey_4096ch_1M")
    nchan, nsamp = w["nchan"], w["nsamp"]
    say(f"survey_4096ch_1M: {nchan} ch x {nsamp}, {len(w['dms'])} DMs")
    pitch = (nsamp + 255) // 256 * 256
    x_host = torch.empty((nchan, pitch), dtype=torch.uint8).pin_memory()
    make_input(w, pitch=pitch, out=x_host.numpy())
    plan = Plan.from_workload(w)
    s = plan.shifts().astype(np.int64)
    assert np.array_equal(s, oracle.shift_table(w["dms"], nchan, w["f_top"], w["foff"], w["tsamp"]))
    info = plan.info
    x = x_host.to("cuda")
    dd = torch.empty((info["ndm"], info["out_pitch"]), dtype=torch.int32, device="cuda")
    return dict(w=w, plan=plan, s=s, info=info, x=x, x_np=x_host.numpy()[:, :nsamp], dd=dd)


def _oracle_samples(x_np, s, d, t):
    """D[d][t] for arrays of (d, t), one sum over channels each."""
    c = np.arange(s.shape[1])
    out = np.empty(len(d), dtype=np.int64)
    for i0 in range(0, len(d), 256):
        dd, tt = d[i0:i0 + 256], t[i0:i0 + 256]
        out[i0:i0 + 256] = x_np[c[None, :], tt[:, None] + s[dd]].astype(np.int64).sum(axis=1)
    return out


def _check_plane(sv, D, rng):
    import torch
    x_np, s, info = sv["x_np"], sv["s"], sv["info"]
    ndm, n_out = info["ndm"], info["n_dd"]
    d = rng.integers(0, ndm, 4000)
    t = rng.integers(0, n_out, 4000)
    cols = [0, n_out - 1, int(rng.integers(0, n_out))]
    d = np.concatenate([d] + [np.arange(ndm)] * len(cols))
    t = np.concatenate([t] + [np.full(ndm, c) for c in cols])
    di = torch.from_numpy(d).cuda()
    ti = torch.from_numpy(t).cuda()
    got = D[di, ti].cpu().numpy().astype(np.int64)
    want = _oracle_samples(x_np, s, d, t)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} sampled outputs differ, first (d, t) = ({d[bad[0]]}, {t[bad[0]]})"
    for dr in (0, int(rng.integers(0, ndm)), ndm - 1):
        t0 = int(rng.integers(0, n_out - 32768))
        want = oracle.dedisperse_rows(x_np[:, t0:t0 + 32768 + int(s.max())], s, [dr])[0]
        got = D[dr, t0:t0 + 32768].cpu().numpy().astype(np.int64)
        assert np.array_equal(got, want), (dr, t0)


def test_survey_dedisp_sampled(survey):
    from paper_2101_00941_amd import Plan
    sv = survey
    plan, x, dd, n_in = sv["plan"], sv["x"], sv["dd"], sv["w"]["nsamp"]
    rng = np.random.default_rng(11)
    ms = plan.autotune(x, n_in=n_in, out=dd, reps=1)
    say(f"  autotune ms per variant {['%.1f' % m for m in ms]} -> variant {plan.variant}")
    chosen = plan.variant
    _check_plane(sv, dd, rng)
    # every matrix-core and quad variant (any of them can be the autotuner's pick, and the
    # quad variants differ in tile, waves and samples per lane), and the first variant of
    # each other layout
    check = {v for v, info in enumerate(Plan.variants()) if info["layout"] in (4, 5, 6, 7)}
    layouts = {}
    for v, info in enumerate(Plan.variants()):
        layouts.setdefault(info["layout"], v)
    check |= set(layouts.values())
    for v in sorted(check - {chosen}):
        say(f"  variant {v}")
        plan.set_variant(v)
        dd.fill_(-1)
        plan.dedisperse(x, n_in=n_in, out=dd)
        _check_plane(sv, dd, rng)
    plan.set_variant(chosen)


def _checked_rows(w, ndm):
    """Every 100th trial, and the two trials on each side of the trial nearest to each
    injected pulse's DM (the rows come from the signal model, not from the GPU list)."""
    dms = np.asarray(w["dms"])
    rows = set(range(0, ndm, 100))
    for p in w["pulses"]:
        r = int(np.argmin(np.abs(dms - p.dm)))
        rows |= {q for q in range(r - 2, r + 3) if 0 <= q < ndm}
    return sorted(rows)


def _runs(rows):
    """Contiguous runs [a, b] of a sorted row list."""
    out = []
    for r in rows:
        if out and r == out[-1][1] + 1:
            out[-1][1] = r
        else:
            out.append([r, r])
    return out


def test_survey_candidates_full_time(survey):
    """GPU candidates over the full time range of the checked rows equal the oracle's,
    which dedisperses each checked row and its two neighbours over all 1,012,255
    samples and runs its own search (statistics, boxcars, peaks) over all starts."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    import torch
    from paper_2101_00941_amd import candidates_as_tuples, candidates_to_numpy
    sv = survey
    w, plan, x, dd, info, s = sv["w"], sv["plan"], sv["x"], sv["dd"], sv["info"], sv["s"]
    n_in, ndm, T, B = w["nsamp"], info["ndm"], info["n_start"], info["stat_block"]
    M = int(s.max())
    plan.dedisperse(x, n_in=n_in, out=dd)
    cap = 1 << 20
    work = torch.empty(plan.work_bytes(T), dtype=torch.uint8, device="cuda")
    cand, count, _ = plan.single_pulse(dd, work=work, cap=cap)
    torch.cuda.synchronize()
    got = candidates_as_tuples(candidates_to_numpy(cand, count))
    say(f"  {len(got)} GPU candidates (variant {plan.variant})")
    assert 0 < len(got) < cap
    rows = _checked_rows(w, ndm)
    need = sorted({q for r in rows for q in (r - 1, r, r + 1) if 0 <= q < ndm})
    say(f"  oracle: {len(rows)} checked rows, {len(need)} dedispersed rows over the full time range")
    x_np = sv["x_np"]

    def one_row(q):
        return q, oracle.dedisperse_rows(x_np, s, [q], n_in, M)[0]

    Drow = {}
    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as pool:
        for q, r in pool.map(one_row, need):
            Drow[q] = r
    want = []
    for a, b in _runs(rows):
        lo, hi = max(a - 1, 0), min(b + 1, ndm - 1)
        D = np.stack([Drow[q] for q in range(lo, hi + 1)])
        c, _ = oracle.single_pulse(D, 0, 0, T, T, w["widths"], w["threshold"], B, row0=lo, ndm=ndm,
                                   report_rows=list(range(a, b + 1)))
        want.extend(c)
    want.sort(key=lambda c: (c[0], c[1]))
    rowset = set(rows)
    have = [c for c in got if c[0] in rowset]
    say(f"  {len(want)} oracle candidates on the checked rows, {len(have)} GPU")
    assert_candidates_equal(have, want)
    # the injected pulses are found at their DM (within two trials) and arrival time
    dms = np.asarray(w["dms"])
    found = 0
    for p in w["pulses"]:
        r = int(np.argmin(np.abs(dms - p.dm)))
        found += any(abs(c[0] - r) <= 2 and abs(c[1] - p.t0) <= 512 for c in want)
    say(f"  {found} of {len(w['pulses'])} injected pulses found")
    assert found >= len(w["pulses"]) - 2


def test_survey_decimated_ranges_rows(survey):
    """Per-range time decimation at the survey size, as the bench runs it (six ranges at
    factors 1..32, the autotuned variant): the GPU candidates of every 100th trial and of the
    trials around each injected pulse equal the oracle's, which decimates the input itself
    (channel blocks of 256, exact halvings), dedisperses those trials and their in-range
    neighbours over the full decimated time range, and searches them per range."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    import torch
    from paper_2101_00941_amd import RangePlan, candidates_as_tuples, candidates_to_numpy
    sv = survey
    w, x, x_np = sv["w"], sv["x"], sv["x_np"]
    first, factor = [0, 512, 1024, 1536, 2048, 2432], [1, 2, 4, 8, 16, 32]
    ndm, nsamp, B = len(w["dms"]), w["nsamp"], w["stat_block"]
    rp = RangePlan(w["nchan"], nsamp, w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"],
                   first, factor, B)
    rp.set_variant(sv["plan"].variant)
    cap = 1 << 20
    cand, count = rp.run(x, n_in=nsamp, cap=cap)
    torch.cuda.synchronize()
    got = candidates_as_tuples(candidates_to_numpy(cand, count))
    assert 0 < len(got) < cap
    say(f"  decimated: {len(got)} GPU candidates (variant {sv['plan'].variant})")
    plans = oracle.range_plans(w["dms"], w["nchan"], nsamp, w["f_top"], w["foff"], w["tsamp"], w["widths"], B,
                               first, factor)
    # decimated inputs, level by level, in channel blocks (bounded temporaries)
    levels = {1: x_np}
    f = 1
    while f < factor[-1]:
        src = levels[f]
        dst = np.empty((src.shape[0], src.shape[1] // 2), dtype=np.uint8)
        for c0 in range(0, src.shape[0], 256):
            dst[c0:c0 + 256] = oracle.decimate2(src[c0:c0 + 256])
        f *= 2
        levels[f] = dst
    checked = set(_checked_rows(w, ndm))
    want, rows_all = [], set()
    jobs = []
    for rp_o in plans:
        lo, hi = rp_o["lo"], rp_o["hi"]
        rows = sorted(r - lo for r in checked if lo <= r < hi)
        if not rows:
            continue
        rows_all |= {lo + r for r in rows}
        need = sorted({q for r in rows for q in (r - 1, r, r + 1) if 0 <= q < hi - lo})
        jobs.append((rp_o, rows, need))
    say(f"  oracle: {len(rows_all)} checked trials over {len(jobs)} ranges")

    def one(args):
        rp_o, q = args
        M = rp_o["sizes"]["maxshift"]
        return rp_o["lo"], q, oracle.dedisperse_rows(levels[rp_o["f"]], rp_o["shifts"], [q], rp_o["n"], M)[0]

    work = [(rp_o, q) for rp_o, rows, need in jobs for q in need]
    D = {}
    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as pool:
        for lo, q, row in pool.map(one, work):
            D[(lo, q)] = row
    for rp_o, rows, need in jobs:
        lo, f, T = rp_o["lo"], rp_o["f"], rp_o["sizes"]["n_start"]
        for a, b in _runs(rows):
            r0, r1 = max(a - 1, 0), min(b + 1, rp_o["hi"] - lo - 1)
            plane = np.stack([D[(lo, q)] for q in range(r0, r1 + 1)])
            c, _ = oracle.single_pulse(plane, 0, 0, T, T, w["widths"], w["threshold"], rp_o["block"], row0=r0,
                                       ndm=rp_o["hi"] - lo, report_rows=list(range(a, b + 1)))
            want.extend((lo + d, f * t, f * wd, s) for d, t, wd, s in c)
    want.sort(key=lambda c: (c[0], c[1]))
    have = [c for c in got if c[0] in rows_all]
    say(f"  {len(want)} oracle candidates on the checked trials, {len(have)} GPU")
    assert len(want) > 0
    assert_candidates_equal(have, want)
