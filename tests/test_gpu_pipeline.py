"""GPU tests of the streamed pipeline (aa_pipeline_*, aa_stream_submit, aa_poll):
chunked and streamed results must equal the whole-signal oracle exactly, for any
number of streams, chunk size and beam mix."""

import numpy as np
import pytest

import oracle
from synth.filterbank import Pulse, make_filterbank
from tests.gpu_util import assert_candidates_equal, say

pytestmark = pytest.mark.gpu

F_TOP, FOFF, TSAMP = 1500.0, 0.78125, 64e-6
WIDTHS = [1, 2, 4, 8, 16, 32]


def _signal(nchan, nsamp, seed, chunk=1 << 17):
    # pulses on chunk edges and on the sub-chunk edges of 2, 4 and 8 streams
    offs = [0, 1, (1 << 15) - 2, 1 << 15, (1 << 16) - 1, 100000 % chunk]
    pulses = [Pulse(50.0, 20000.0, 4.0, 48.0)]
    for k in range(1, nsamp // chunk):
        pulses.append(Pulse(20.0 + 7 * k, float(k * chunk + offs[k % len(offs)]), 4.0, 48.0))
    return make_filterbank(nchan, nsamp, F_TOP, FOFF, TSAMP, pulses, seed=seed)


@pytest.fixture(scope="module")
def sig():
    import torch
    nchan, nsamp = 128, 1 << 19
    dms = np.arange(0, 100, 1.0)
    x = _signal(nchan, nsamp, seed=31)
    want = oracle.run(x, nsamp, F_TOP, FOFF, TSAMP, dms, WIDTHS, 6.0, stat_block=32768)["candidates"]
    host = torch.from_numpy(np.ascontiguousarray(x)).pin_memory()
    return dict(x=x, host=host, pageable=np.ascontiguousarray(x), nchan=nchan, nsamp=nsamp, dms=dms, want=want)


def _run(sig, chunk, nstreams, serial=False, cap=1 << 14, sdma=False, staged=False, pageable=False, min_piece_work=-1):
    """min_piece_work -1 (the default here) splits every chunk over all streams, as the
    paper does, so that the sub-chunk edges are exercised at these small sizes."""
    from paper_2101_00941_amd import Pipeline, Plan
    plan = Plan(sig["nchan"], sig["nsamp"], F_TOP, FOFF, TSAMP, sig["dms"], WIDTHS, 6.0, 32768)
    pipe = Pipeline(nstreams=nstreams, max_beams=1, max_chunk=chunk, cand_cap=cap, hbm_budget=2 << 30,
                    serial=serial, timing=True, sdma_copy=sdma, staged=staged, min_piece_work=min_piece_work)
    b = pipe.add_beam(plan)
    host, nsamp = (sig["pageable"] if pageable else sig["host"]), sig["nsamp"]
    tags = []
    for k, a in enumerate(range(0, nsamp, chunk)):
        n = min(chunk, nsamp - a)
        pitch = host.strides[0] if pageable else host.stride(0)
        pipe.submit(b, host[:, a:a + n], nsamp=n, pitch=pitch, tag=k, last=(a + n == nsamp))
        tags.append(k)
    got, seen, covered = [], set(), []
    while len(seen) < len(tags):
        r = pipe.poll(timeout_us=20_000_000)
        assert r is not None, "pipeline stalled"
        assert r["status"] == 0, r
        seen.add(r["tag"])
        covered.append((r["t_begin"], r["t_end"]))
        got.extend((int(c["dm_idx"]), int(c["t"]), int(c["width"]), float(c["snr"])) for c in r["cand"])
    st = pipe.stats()
    pipe.close()
    got.sort(key=lambda c: (c[0], c[1]))
    return got, sorted(covered), st


@pytest.mark.parametrize("nstreams,serial", [(1, True), (1, False), (2, False), (4, False), (8, False)])
def test_streamed_equals_whole_signal(sig, nstreams, serial):
    say(f"pipeline nstreams={nstreams} serial={serial}")
    got, covered, st = _run(sig, 1 << 17, nstreams, serial)
    assert_candidates_equal(got, sig["want"])
    T = sig["nsamp"] - 418 - 32 + 1
    # consecutive chunks cover [0, T) exactly once
    pos = 0
    for a, b in covered:
        assert a == pos
        pos = b
    assert pos == T
    assert st["completed"] == st["submitted"] and st["in_flight"] == 0 and st["arena_used"] > 0
    say(f"  copy {st['copy_ms']:.2f} ms, kernels {st['kernel_ms']:.2f} ms, overlap {st['overlap_ms']:.2f} ms")


@pytest.mark.parametrize("chunk", [100_000, 40_000, 250_000, 99_999])
def test_odd_chunk_sizes(sig, chunk):
    got, _, _ = _run(sig, chunk, 4)
    assert_candidates_equal(got, sig["want"])


def test_runtime_copy_path_matches(sig):
    got, _, _ = _run(sig, 1 << 17, 2, sdma=True)
    assert_candidates_equal(got, sig["want"])


@pytest.mark.parametrize("nstreams,chunk,staged", [(1, 1 << 17, False), (4, 1 << 17, True), (3, 99_999, True),
                                                   (8, 40_000, True)])
def test_pageable_input_matches(sig, nstreams, chunk, staged):
    """Pageable host input: staged through the runtime, or through the pipeline's pinned
    bounce buffers and stage threads; the result equals the whole-signal oracle."""
    say(f"pageable input nstreams={nstreams} chunk={chunk} staged={staged}")
    got, covered, st = _run(sig, chunk, nstreams, staged=staged, pageable=True)
    assert_candidates_equal(got, sig["want"])
    assert st["completed"] == st["submitted"]


def test_multi_beam_mix_equals_alone():
    """Three beams with different plans, chunks interleaved: each beam's result in the
    mix equals its own whole-signal oracle result (and so its result alone)."""
    import torch
    from paper_2101_00941_amd import Pipeline, Plan
    beams = []
    for i, (nchan, ndm, nsamp) in enumerate([(64, 40, 300_000), (128, 100, 262_144), (96, 70, 400_000)]):
        x = _signal(nchan, nsamp, seed=40 + i, chunk=1 << 16)
        dms = np.arange(ndm) * 1.5
        want = oracle.run(x, nsamp, F_TOP, FOFF, TSAMP, dms, WIDTHS, 6.0, stat_block=16384)["candidates"]
        beams.append(dict(x=x, host=torch.from_numpy(np.ascontiguousarray(x)).pin_memory(), nchan=nchan,
                          nsamp=nsamp, dms=dms, want=want))
    pipe = Pipeline(nstreams=4, max_beams=3, max_chunk=90_000, cand_cap=1 << 14, hbm_budget=3 << 30)
    ids = []
    for bd in beams:
        bd["plan"] = Plan(bd["nchan"], bd["nsamp"], F_TOP, FOFF, TSAMP, bd["dms"], WIDTHS, 6.0, 16384)
        ids.append(pipe.add_beam(bd["plan"]))
    rng = np.random.default_rng(0)
    pos = [0, 0, 0]
    tag = 0
    expect = 0
    while any(pos[i] < beams[i]["nsamp"] for i in range(3)):
        i = int(rng.integers(0, 3))
        bd = beams[i]
        if pos[i] >= bd["nsamp"]:
            continue
        n = min(int(rng.integers(20_000, 90_001)), bd["nsamp"] - pos[i])
        pipe.submit(ids[i], bd["host"][:, pos[i]:pos[i] + n], nsamp=n, pitch=bd["host"].stride(0), tag=tag,
                    last=pos[i] + n == bd["nsamp"])
        pos[i] += n
        tag += 1
        expect += 1
    got = {i: [] for i in range(3)}
    for _ in range(expect):
        r = pipe.poll(timeout_us=20_000_000)
        assert r is not None and r["status"] == 0
        got[r["beam"]].extend((int(c["dm_idx"]), int(c["t"]), int(c["width"]), float(c["snr"])) for c in r["cand"])
        assert all(int(c["beam"]) == r["beam"] for c in r["cand"])
    pipe.close()
    for i in range(3):
        g = sorted(got[i], key=lambda c: (c[0], c[1]))
        assert_candidates_equal(g, beams[i]["want"])


def test_pipeline_argument_errors():
    from paper_2101_00941_amd import AAError, Pipeline, Plan
    with pytest.raises(AAError):
        Pipeline(nstreams=0)
    with pytest.raises(AAError):
        Pipeline(nstreams=2, hbm_budget=0)
    pipe = Pipeline(nstreams=2, max_beams=1, max_chunk=1 << 16, hbm_budget=64 << 20)
    plan = Plan(64, 1 << 20, F_TOP, FOFF, TSAMP, np.arange(10.0), WIDTHS, 6.0)
    b = pipe.add_beam(plan)
    with pytest.raises(AAError):
        pipe.add_beam(plan)                                    # max_beams reached
    import torch
    host = torch.zeros((64, 1 << 17), dtype=torch.uint8).pin_memory()
    with pytest.raises(AAError):
        pipe.submit(b, host, nsamp=1 << 17, tag=1)             # larger than max_chunk
    with pytest.raises(AAError):
        pipe.submit(7, host, nsamp=100, tag=2)                 # unknown beam
    pipe.submit(b, host[:, :1000], nsamp=1000, pitch=host.stride(0), tag=3)
    with pytest.raises(AAError):
        pipe.submit(b, host[:, :1000], nsamp=1000, pitch=host.stride(0), tag=3)   # tag in use
    r = pipe.poll(timeout_us=10_000_000)
    assert r is not None and r["t_begin"] == r["t_end"] == 0 and len(r["cand"]) == 0
    assert pipe.poll(timeout_us=0) is None
    pipe.close()


def test_hbm_budget_too_small_for_beam():
    from paper_2101_00941_amd import AAError, Pipeline, Plan
    pipe = Pipeline(nstreams=1, max_beams=1, max_chunk=1 << 20, hbm_budget=16 << 20)
    plan = Plan(4096, 1 << 21, 1450.0, 300.0 / 4096, 64e-6, np.arange(10.0), WIDTHS, 6.0)
    with pytest.raises(AAError) as e:
        pipe.add_beam(plan)
    assert e.value.code == -3
    pipe.close()


@pytest.mark.parametrize("nstreams", [4, 8])
def test_default_split_policy_matches(sig, nstreams):
    """The default sub-chunk policy (no piece below 2^33 trial x channel x start units)
    keeps these small chunks whole and spreads consecutive chunks over the streams."""
    got, covered, st = _run(sig, 1 << 17, nstreams, min_piece_work=0)
    assert_candidates_equal(got, sig["want"])


def test_injected_fault_surfaces_on_its_tag(sig, tmp_path, monkeypatch):
    """AA_FAULT=unit:K (read at create) skips the launch of the K-th sub-chunk: exactly
    that chunk reports AA_EHIP on aa_poll, every other chunk's candidates are exact, and
    AA_LOG records one line per chunk with its status. No kernel is faulted: the skipped
    sub-chunk simply launches nothing."""
    import json

    from paper_2101_00941_amd import Pipeline, Plan
    log = tmp_path / "chunks.jsonl"
    monkeypatch.setenv("AA_FAULT", "unit:2")
    monkeypatch.setenv("AA_LOG", str(log))
    plan = Plan(sig["nchan"], sig["nsamp"], F_TOP, FOFF, TSAMP, sig["dms"], WIDTHS, 6.0, 32768)
    pipe = Pipeline(nstreams=2, max_beams=1, max_chunk=1 << 17, hbm_budget=2 << 30, min_piece_work=-1)
    monkeypatch.delenv("AA_FAULT")
    monkeypatch.delenv("AA_LOG")
    b = pipe.add_beam(plan)
    host, nsamp, chunk = sig["host"], sig["nsamp"], 1 << 17
    n = 0
    for k, a in enumerate(range(0, nsamp, chunk)):
        m = min(chunk, nsamp - a)
        pipe.submit(b, host[:, a:a + m], nsamp=m, pitch=host.stride(0), tag=k, last=(a + m == nsamp))
        n += 1
    bad, good = [], []
    for _ in range(n):
        r = pipe.poll(timeout_us=20_000_000)
        assert r is not None
        if r["status"] != 0:
            assert r["status"] == -4
            bad.append((r["t_begin"], r["t_end"]))
        else:
            good.extend((int(c["dm_idx"]), int(c["t"]), int(c["width"]), float(c["snr"])) for c in r["cand"])
    pipe.close()
    assert len(bad) == 1
    lo, hi = bad[0]
    want = [c for c in sig["want"] if not lo <= c[1] < hi]
    good = sorted((c for c in good if not lo <= c[1] < hi), key=lambda c: (c[0], c[1]))
    assert_candidates_equal(good, want)
    lines = [json.loads(x) for x in log.read_text().splitlines()]
    assert len(lines) == n and sum(1 for x in lines if x["status"] == -4) == 1


@pytest.mark.parametrize("cut_chunks", [1, 2])
def test_checkpoint_resume_equals_uninterrupted(sig, cut_chunks):
    """Stop a beam after some chunks and destroy its pipeline; a new pipeline resumes at
    the last t_end (aa_pipeline_add_beam_at) with the samples from the resume column on.
    The concatenated candidates equal the whole-signal oracle."""
    from paper_2101_00941_amd import Pipeline, Plan
    plan = Plan(sig["nchan"], sig["nsamp"], F_TOP, FOFF, TSAMP, sig["dms"], WIDTHS, 6.0, 32768)
    host, nsamp, chunk = sig["host"], sig["nsamp"], 100_000
    got, ckpt = [], 0
    pipe = Pipeline(nstreams=2, max_beams=1, max_chunk=chunk, hbm_budget=2 << 30)
    b = pipe.add_beam(plan)
    for k in range(cut_chunks):
        pipe.submit(b, host[:, k * chunk:(k + 1) * chunk], nsamp=chunk, pitch=host.stride(0), tag=k)
    for _ in range(cut_chunks):
        r = pipe.poll(timeout_us=20_000_000)
        assert r is not None and r["status"] == 0
        ckpt = max(ckpt, r["t_end"])
        got.extend((int(c["dm_idx"]), int(c["t"]), int(c["width"]), float(c["snr"])) for c in r["cand"])
    pipe.close()
    assert ckpt > 0 and ckpt % 32768 == 0
    pipe = Pipeline(nstreams=3, max_beams=1, max_chunk=chunk, hbm_budget=2 << 30)
    b = pipe.add_beam(plan, t_resume=ckpt)
    a = (ckpt - 1) & ~15
    tag, n = 100, 0
    while a < nsamp:
        m = min(chunk, nsamp - a)
        pipe.submit(b, host[:, a:a + m], nsamp=m, pitch=host.stride(0), tag=tag, last=(a + m == nsamp))
        a, tag, n = a + m, tag + 1, n + 1
    first = None
    for _ in range(n):
        r = pipe.poll(timeout_us=20_000_000)
        assert r is not None and r["status"] == 0
        first = r["t_begin"] if first is None else min(first, r["t_begin"])
        got.extend((int(c["dm_idx"]), int(c["t"]), int(c["width"]), float(c["snr"])) for c in r["cand"])
    pipe.close()
    assert first == ckpt
    got.sort(key=lambda c: (c[0], c[1]))
    assert_candidates_equal(got, sig["want"])
