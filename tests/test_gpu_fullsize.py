"""Parity at the survey size: 4096 channels x 2^20 samples, 3000 DM trials (doubling
steps to DM 1998), boxcars 1..256, threshold 6, in the configuration the benchmark
times (resident input, one stream, autotuned dedispersion variant).

The whole plane (3000 x 1,012,255 int32, 12 GB) is beyond the oracle, so the
oracle checks sampled outputs, each computed on its own:
  * dedispersion: random (trial, sample) pairs, every trial at the first and last
    samples and at a random one, and full 32768-sample runs of a few trials, for
    the autotuned variant, every matrix-core variant and one variant of each other
    kernel family;
  * candidates: regions of one trial x one statistics block, where the oracle
    dedisperses the trial and its two neighbours over the block (plus boxcar and
    peak halo) and runs its own search. Regions are those of the strongest GPU
    candidates and a few random ones. The GPU list restricted to the region must
    equal the oracle's exactly.
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
    # every matrix-core variant (any of them can be the autotuner's pick), and the first
    # variant of each other layout
    check = {v for v, info in enumerate(Plan.variants()) if info["layout"] in (4, 5, 6)}
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


def test_survey_candidates_regions(survey):
    import torch
    sv = survey
    w, plan, x, dd, info, s = sv["w"], sv["plan"], sv["x"], sv["dd"], sv["info"], sv["s"]
    n_in, ndm, T, B = w["nsamp"], info["ndm"], info["n_start"], info["stat_block"]
    M, wmax = int(s.max()), max(w["widths"])
    plan.dedisperse(x, n_in=n_in, out=dd)
    cap = 1 << 20
    work = torch.empty(plan.work_bytes(T), dtype=torch.uint8, device="cuda")
    cand, count, _ = plan.single_pulse(dd, work=work, cap=cap)
    torch.cuda.synchronize()
    from paper_2101_00941_amd import candidates_as_tuples, candidates_to_numpy
    got = candidates_as_tuples(candidates_to_numpy(cand, count))
    say(f"  {len(got)} GPU candidates")
    assert 0 < len(got) < cap
    rng = np.random.default_rng(12)
    top = sorted(got, key=lambda c: -c[3])[:10]
    regions = {(c[0], c[1] // B) for c in top}
    regions |= {(int(rng.integers(0, ndm)), int(rng.integers(0, (T + B - 1) // B))) for _ in range(3)}
    regions |= {(0, 0), (ndm - 1, (T - 1) // B)}
    x_np = sv["x_np"]
    for r, blk in sorted(regions):
        b0, b1 = blk * B, min(blk * B + B, T)
        lo = max(b0 - 1, 0)
        hi_start = b1 + 1 if b1 + 1 <= T else T               # starts the peak test can touch
        cols = hi_start + wmax - 1 - lo                          # plane columns those starts need
        rows = [q for q in (r - 1, r, r + 1) if 0 <= q < ndm]
        Dr = oracle.dedisperse_rows(x_np[:, lo:lo + cols + M], s, rows, maxshift=M)
        want, _ = oracle.single_pulse(Dr, lo, b0, b1, T, w["widths"], w["threshold"], B, row0=rows[0], ndm=ndm,
                                      report_rows=[r])
        have = [c for c in got if c[0] == r and b0 <= c[1] < b1]
        say(f"  region trial {r} starts [{b0}, {b1}): {len(want)} candidates")
        assert_candidates_equal(have, want)
