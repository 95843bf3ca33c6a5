"""GPU tests of aa_batch_run: beams of uneven shape in one persistent launch must give
exactly the per-beam plain results (aa_dedisperse + aa_single_pulse), and the oracle's."""

import numpy as np
import pytest

import oracle
from synth.filterbank import Pulse, make_filterbank
from tests.gpu_util import assert_candidates_equal, run_gpu, say, to_device

pytestmark = pytest.mark.gpu

WIDTHS = [1, 2, 4, 8, 16]


def _beams():
    shapes = [(64, 60_000, 40), (96, 90_000, 77), (128, 50_000, 100), (48, 120_000, 33), (80, 70_001, 60)]
    out = []
    for i, (nchan, nsamp, ndm) in enumerate(shapes):
        foff = 1.0
        dms = np.arange(ndm) * 1.25
        pulses = [Pulse(float(dms[ndm // 2]), nsamp * 0.4, 3.0, 60.0), Pulse(float(dms[ndm // 3]), nsamp * 0.7, 6.0, 40.0)]
        x = make_filterbank(nchan, nsamp, 1500.0, foff, 64e-6, pulses, seed=70 + i)
        out.append(dict(nchan=nchan, nsamp=nsamp, dms=dms, x=x, foff=foff))
    return out


@pytest.fixture(scope="module")
def beams():
    from paper_2101_00941_amd import Plan
    bs = _beams()
    for b in bs:
        b["plan"] = Plan(b["nchan"], b["nsamp"], 1500.0, b["foff"], 64e-6, b["dms"], WIDTHS, 6.0, 8192)
        b["dev"] = to_device(b["x"], b["nsamp"])
    return bs


@pytest.mark.parametrize("static", [False, True])
@pytest.mark.parametrize("work_mb", [512, 40])          # 40 MB forces several groups
def test_batch_equals_plain_per_beam(beams, static, work_mb):
    from paper_2101_00941_amd import batch_run, candidates_as_tuples
    say(f"batch static={static} work={work_mb} MB")
    cands, counts, info = batch_run([(b["plan"], b["dev"], b["nsamp"]) for b in beams], variant=1,
                                    work_bytes=work_mb << 20, cap=4096, static=static)
    if work_mb == 40:
        assert info["groups"] > 1
    for i, b in enumerate(beams):
        plain = run_gpu(b["plan"], b["x"], b["nsamp"], cap=4096, want_best=False)
        got = candidates_as_tuples(cands[i])
        assert counts[i] == plain["count"]
        assert_candidates_equal(got, plain["candidates"])
        assert all(int(c["beam"]) == i for c in cands[i])


def test_batch_matches_oracle_and_autotunes(beams):
    from paper_2101_00941_amd import batch_run, candidates_as_tuples
    cands, counts, info = batch_run([(b["plan"], b["dev"], b["nsamp"]) for b in beams], variant=-1,
                                    work_bytes=512 << 20, cap=4096)
    say(f"batch info {info}")
    assert 0 <= info["variant"] < 6 and info["items"] > 0
    for i in (0, 3):
        b = beams[i]
        want = oracle.run(b["x"], b["nsamp"], 1500.0, b["foff"], 64e-6, b["dms"], WIDTHS, 6.0, stat_block=8192)
        assert_candidates_equal(candidates_as_tuples(cands[i]), want["candidates"])
        assert counts[i] == len(want["candidates"])


def test_batch_errors(beams):
    from paper_2101_00941_amd import AAError, batch_run
    with pytest.raises(AAError):
        batch_run([(b["plan"], b["dev"], b["nsamp"]) for b in beams], variant=1, work_bytes=1 << 20, cap=16)
