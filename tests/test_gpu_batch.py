"""GPU tests of aa_batch_run: beams of uneven shape in one persistent launch must give
exactly the per-beam plain results (aa_dedisperse + aa_single_pulse), and the oracle's.

The beams differ in channel count (some not a multiple of the 4 or 8 channels of a
matrix-core step, so those kernels pad), length (some not a multiple of a time tile)
and DM plan. A small work buffer forces several groups, i.e. several persistent
launches, each with a different mix of beams."""

import numpy as np
import pytest

import oracle
from synth.filterbank import Pulse, make_filterbank
from tests.gpu_util import assert_candidates_equal, run_gpu, say, to_device

pytestmark = pytest.mark.gpu

WIDTHS = [1, 2, 4, 8, 16]
# (nchan, nsamp, ndm): 70 and 33 channels are padded by the matrix-core kernels
SHAPES = [(64, 60_000, 40), (96, 90_000, 77), (128, 50_000, 100), (48, 120_000, 33), (80, 70_001, 60),
          (70, 65_003, 50), (33, 40_000, 25)]


def _beams():
    out = []
    for i, (nchan, nsamp, ndm) in enumerate(SHAPES):
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


@pytest.fixture(scope="module")
def want(beams):
    """The oracle's candidate list for every beam (whole signal)."""
    return [oracle.run(b["x"], b["nsamp"], 1500.0, b["foff"], 64e-6, b["dms"], WIDTHS, 6.0,
                       stat_block=8192)["candidates"] for b in beams]


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
        b["plan"].set_variant(1)
        plain = run_gpu(b["plan"], b["x"], b["nsamp"], cap=4096, want_best=False)
        got = candidates_as_tuples(cands[i])
        assert counts[i] == plain["count"]
        assert_candidates_equal(got, plain["candidates"])
        assert all(int(c["beam"]) == i for c in cands[i])


@pytest.mark.parametrize("variant", [12, 17, 20, 14, 16, 21, 22, 23, 24])
@pytest.mark.parametrize("work_mb", [512, 40])
def test_batch_matrix_core_and_quad_variants_match_oracle(beams, want, variant, work_mb):
    """The persistent matrix-core kernels (one step shape, the mixed shape, and the
    two-work-group-per-CU variants whose batch kernels spill registers) and the quad
    shift-and-add kernels (whose batch kernels spill too) against the oracle, every
    beam, with one group and with several."""
    from paper_2101_00941_amd import batch_run, candidates_as_tuples
    say(f"batch variant {variant} work={work_mb} MB")
    cands, counts, info = batch_run([(b["plan"], b["dev"], b["nsamp"]) for b in beams], variant=variant,
                                    work_bytes=work_mb << 20, cap=4096)
    assert info["variant"] == variant and info["items"] > 0
    if work_mb == 40:
        assert info["groups"] > 1
    for i in range(len(beams)):
        assert counts[i] == len(want[i]), (i, counts[i], len(want[i]))
        assert_candidates_equal(candidates_as_tuples(cands[i]), want[i])
        assert all(int(c["beam"]) == i for c in cands[i])


def test_batch_autotune_picks_fastest_and_matches_oracle(beams, want):
    from paper_2101_00941_amd import batch_run, candidates_as_tuples
    cands, counts, info = batch_run([(b["plan"], b["dev"], b["nsamp"]) for b in beams], variant=-1,
                                    work_bytes=512 << 20, cap=4096)
    ms = info["tune_ms"]
    say(f"batch autotune on beam {info['tuned_beam']}: variant {info['variant']}, ms {['%.3f' % m for m in ms]}")
    timed = [(m, v) for v, m in enumerate(ms) if m >= 0]
    assert timed, "the autotuner timed no variant"
    assert info["variant"] == min(timed)[1]
    sizes = [b["plan"].info["ndm"] * b["plan"].info["n_dd"] * b["nchan"] for b in beams]
    assert info["tuned_beam"] == int(np.argmax(sizes))
    for i in range(len(beams)):
        assert_candidates_equal(candidates_as_tuples(cands[i]), want[i])
        assert counts[i] == len(want[i])


def test_batch_errors(beams):
    from paper_2101_00941_amd import AAError, batch_run
    with pytest.raises(AAError):
        batch_run([(b["plan"], b["dev"], b["nsamp"]) for b in beams], variant=1, work_bytes=1 << 20, cap=16)
