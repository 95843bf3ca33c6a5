"""GPU parity of per-range time decimation (aa_decimate2, aa_range_plan, aa_range_run)
against the oracle: the halving bit for bit on ragged rows, and the candidate list of a
multi-range plan (factors 1, 2, 4, 8) exactly, including a truncated list."""

import numpy as np
import pytest

import oracle
from synth.dmplan import dm_plan
from synth.filterbank import Pulse, make_filterbank
from tests.gpu_util import assert_candidates_equal, say, to_device

pytestmark = pytest.mark.gpu

F_TOP, TSAMP = 1450.0, 64e-6
WIDTHS = [1, 2, 4, 8, 16, 32]


@pytest.mark.parametrize("nchan,n", [(3, 33), (17, 4096), (64, 100_003), (5, 2)])
def test_decimate2_matches_oracle(nchan, n):
    import torch
    from paper_2101_00941_amd import decimate2
    rng = np.random.default_rng(n)
    x = rng.integers(0, 256, (nchan, n), dtype=np.uint8)
    xd = to_device(x, n, fill=255)
    y = decimate2(xd, n_in=n)
    torch.cuda.synchronize()
    assert np.array_equal(y[:, :n // 2].cpu().numpy(), oracle.decimate2(x))


@pytest.fixture(scope="module")
def case():
    nchan, nsamp = 64, (1 << 16) + 333
    foff = 300.0 / nchan
    dms = dm_plan(600)
    first, factor = [0, 200, 350, 500], [1, 2, 4, 8]
    pulses = [Pulse(float(dms[100]), 20000.0, 3.0, 40.0), Pulse(float(dms[420]), 30000.0, 12.0, 30.0),
              Pulse(float(dms[560]), 45000.0, 24.0, 30.0)]
    x = make_filterbank(nchan, nsamp, F_TOP, foff, TSAMP, pulses, seed=21)
    want = oracle.run_ranges(x, nsamp, F_TOP, foff, TSAMP, dms, WIDTHS, 6.0, 8192, first, factor)
    return dict(x=x, nchan=nchan, nsamp=nsamp, foff=foff, dms=dms, first=first, factor=factor, want=want)


@pytest.mark.parametrize("variant", [12, 20, 1])
def test_range_run_matches_oracle(case, variant):
    import torch
    from paper_2101_00941_amd import RangePlan, candidates_as_tuples, candidates_to_numpy
    c = case
    rp = RangePlan(c["nchan"], c["nsamp"], F_TOP, c["foff"], TSAMP, c["dms"], WIDTHS, 6.0, c["first"], c["factor"], 8192)
    rp.set_variant(variant)
    xd = to_device(c["x"], c["nsamp"])
    cand, count = rp.run(xd, n_in=c["nsamp"], cap=1 << 14)
    torch.cuda.synchronize()
    got = candidates_as_tuples(candidates_to_numpy(cand, count))
    want = c["want"]["candidates"]
    say(f"ranges variant {variant}: {len(got)} candidates, oracle {len(want)}")
    assert int(count.item()) == len(want) and len(want) > 0
    assert_candidates_equal(got, want)
    # every range found its pulse (each range reports starts and widths in input samples)
    for r, f in zip(c["first"][1:], c["factor"][1:]):
        assert all(t % f == 0 and w % f == 0 for d, t, w, _ in got if d >= r)


def test_range_run_truncated_list(case):
    import torch
    from paper_2101_00941_amd import RangePlan, candidates_as_tuples, candidates_to_numpy
    c = case
    rp = RangePlan(c["nchan"], c["nsamp"], F_TOP, c["foff"], TSAMP, c["dms"], WIDTHS, 6.0, c["first"], c["factor"], 8192)
    xd = to_device(c["x"], c["nsamp"])
    want = c["want"]["candidates"]
    cap = len(want) // 2
    cand, count = rp.run(xd, n_in=c["nsamp"], cap=cap)
    torch.cuda.synchronize()
    assert int(count.item()) == len(want)
    got = candidates_as_tuples(candidates_to_numpy(cand, cap, cap))
    assert_candidates_equal(got, want[:cap])


def test_range_plan_errors(case):
    from paper_2101_00941_amd import AAError, RangePlan
    c = case
    args = (c["nchan"], c["nsamp"], F_TOP, c["foff"], TSAMP, c["dms"], WIDTHS, 6.0)
    with pytest.raises(AAError):
        RangePlan(*args, [1, 200], [1, 2])             # does not start at trial 0
    with pytest.raises(AAError):
        RangePlan(*args, [0, 200], [2, 1])             # factors decrease
    with pytest.raises(AAError):
        RangePlan(*args, [0, 200], [1, 3])             # not a power of two
    with pytest.raises(AAError):
        RangePlan(*args, [0, 700], [1, 2])             # first trial past ndm


def test_range_autotune_picks_per_range_and_matches_oracle(case):
    import torch
    from paper_2101_00941_amd import RangePlan, candidates_as_tuples, candidates_to_numpy
    c = case
    rp = RangePlan(c["nchan"], c["nsamp"], F_TOP, c["foff"], TSAMP, c["dms"], WIDTHS, 6.0, c["first"], c["factor"], 8192)
    xd = to_device(c["x"], c["nsamp"])
    chosen = rp.autotune(xd, n_in=c["nsamp"], reps=1)
    say(f"range autotune: {chosen}")
    for r, v in enumerate(chosen):
        timed = [(m, k) for k, m in enumerate(rp.tune_ms[r]) if m >= 0]
        assert v == min(timed)[1]
    cand, count = rp.run(xd, n_in=c["nsamp"], cap=1 << 14)
    torch.cuda.synchronize()
    assert_candidates_equal(candidates_as_tuples(candidates_to_numpy(cand, count)), c["want"]["candidates"])
