"""Benchmark: brute-force dedispersion + single-pulse search on one MI355X.

Default workload: survey_4096ch_1M. That is 4096 channels x 2^20 uint8 samples,
3000 DM trials of the doubling-step plan (0..1998), boxcars 1..256 and threshold 6.
The input is resident in HBM. One step is the whole hot path over that input:
aa_dedisperse (all trials, every sample), then aa_single_pulse (block statistics,
boxcar S/N, 3x3 peaks and ordered candidates), then the asynchronous copy of the
candidate count and list to pinned host memory.

Prints ONE JSON line with the metric, a roofline object for the dominant kernel
(dedispersion, measured with HIP events on its own stream), the best shift-and-add
(no matrix core) variant beside it, the CPU oracle timed on a bounded sample of the
same workload, and two compact sub-objects for the rest of the metric:
  streamed  the streamed pipeline (pinned host input in 2^18-sample chunks) against
            the plain single-stream path: hidden-transfer fraction H, efficiency E and
            wall time per stream count, on the 128-channel signal and on the survey
            signal (16 chunks), with the streamed survey's candidates checked against
            the resident run's;
  serving   32 beams with Poisson arrivals at 1x and 4x real time: p50/p99 chunk
            latency and throughput of continuous batching against the plain FIFO path.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
       python bench.py --mode streamed|serving|batched   (the full runs of each form)
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks used for the roofline object.
HBM_PEAK_GBS = 8000.0
CU, CLOCK_GHZ, LANES = 256, 2.4, 64
# int32 VALU adds: 256 CU x 64 lanes x 2.4 GHz = 39.3 T/s. The kernel adds bytes as
# packed 16-bit pairs inside 32-bit adds, i.e. 2 byte-adds per lane operation.
ALU_PEAK_TOPS = 2 * CU * LANES * CLOCK_GHZ / 1000.0   # 78.6 T byte-adds/s
# LDS read bandwidth: 128 bytes per clock per CU (256 x 128 x 2.4 GHz = 78.6 TB/s). A
# sum that reads each staged byte from LDS once per add is bound there at 1 byte/add.
LDS_PEAK_TBS = CU * 128 * CLOCK_GHZ / 1000.0
# v_sad_u8 adds four bytes per lane operation: 157 T byte-adds/s.
SAD_PEAK_TOPS = 4 * CU * LANES * CLOCK_GHZ / 1000.0
# Dense int8 matrix-core peak (v_mfma_i32_*_i8), TOP/s.
I8_MFMA_PEAK_TOPS = 5000.0
# HBM bytes per launch of the dedispersion kernel (FETCH_SIZE x 2.000 + WRITE_SIZE x
# 1.000 per dispatch, scaled by a 1 GiB copy), from the counter runs summarised in
# profiles/dedisp_*_survey_4096ch_1M.md. Keyed by (workload, variant), with the digest of
# the kernel sources the counters were taken on: after any change to those sources the
# entry no longer matches and the bench reports traffic as null.
TRAFFIC_BYTES = {
    ("survey_4096ch_1M", 20): (196.62e9 + 12.15e9, "2a64072bc06edccd"),
    ("survey_4096ch_1M", 23): (466.86e9 + 12.15e9, "2a64072bc06edccd"),
}
KERNEL_SOURCES = ("dedisp.hip", "tiling.cpp", "aa_internal.h", "xcd.h")
# the part of aa_internal.h that the dedispersion kernels use: tiling constants, variant
# and table layouts, launch arguments
INTERNAL_SPAN = ("// Dedispersion tiling.", "// Single-pulse-search tiling")


def kernel_digest():
    """sha256 (16 hex digits) of the dedispersion kernel sources with comments and blank
    space removed, so that comment edits keep a counter entry valid and code edits do not."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2101_00941_amd", "csrc", name)) as f:
            text = f.read()
        if name == "aa_internal.h":
            text = text[text.index(INTERNAL_SPAN[0]):text.index(INTERNAL_SPAN[1])]
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        h.update(re.sub(r"\s+", " ", text).strip().encode())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, x, threads=None, groups=None, rows_per_group=4):
    """Time the oracle (as it is) on a bounded sample of the workload, on the host's cores.

    The sample is `groups` runs of `rows_per_group` consecutive DM trials, spread evenly
    over the plan. Each run dedisperses its trials and the two neighbour trials (the 3x3
    peak test needs them) over the full time range, then searches its trials over every
    start. Phase 1 times all dedispersion rows in a thread pool, phase 2 all searches
    (numpy releases the GIL in its large operations; threads, since no process may fork
    after the GPU is initialised). Reported:
      dedisp_rate  dedispersed rows x samples / phase-1 wall time
      search_rate  searched rows x starts / phase-2 wall time
      value        the whole plan's rate on these cores when every trial is dedispersed
                   once and searched once: N_dd / (t_dd per row + t_search per row)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    ncpu = os.cpu_count() or 1
    threads = threads or max(1, min(16, ncpu))
    groups = groups or 2 * threads   # about 10 s on 16 host threads
    ndm = len(w["dms"])
    step = ndm // groups
    starts = [min(max(1, step // 2 + k * step), ndm - rows_per_group - 1) for k in range(groups)]
    s = oracle.shift_table(w["dms"], w["nchan"], w["f_top"], w["foff"], w["tsamp"])
    sz = oracle.sizes(s, w["nsamp"], w["widths"], w["stat_block"])
    rows = sorted({r for a in starts for r in range(a - 1, a + rows_per_group + 1)})

    def dd_row(r):
        return r, oracle.dedisperse_rows(x, s, [r], w["nsamp"], sz["maxshift"])[0]

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as pool:
        D = dict(pool.map(dd_row, rows))
    t_dd = time.perf_counter() - t0

    def search(a):
        lo = a - 1
        plane = np.stack([D[r] for r in range(lo, a + rows_per_group + 1)])
        oracle.single_pulse(plane, 0, 0, sz["n_start"], sz["n_start"], w["widths"], w["threshold"], w["stat_block"],
                            row0=lo, ndm=ndm, report_rows=list(range(a, a + rows_per_group)))

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as pool:
        list(pool.map(search, starts))
    t_sps = time.perf_counter() - t0
    n_dd_rows, n_sps_rows = len(rows), groups * rows_per_group
    per_row = t_dd / n_dd_rows + t_sps / n_sps_rows
    return dict(value=sz["n_dd"] / per_row, unit="DM-trial*samples/s", cores=threads, kind="oracle",
                dedisp_rate=n_dd_rows * sz["n_dd"] / t_dd, search_rate=n_sps_rows * sz["n_start"] / t_sps,
                host_cpus=ncpu, cpu_model=_cpu_model(),
                sample=f"{groups} runs of {rows_per_group} consecutive DM trials spread over the plan (first trials "
                       f"{starts[0]}..{starts[-1]}); {n_dd_rows} trials dedispersed (runs plus neighbours) x "
                       f"{sz['n_dd']} samples in {t_dd:.1f} s, {n_sps_rows} trials searched x {sz['n_start']} starts in "
                       f"{t_sps:.1f} s; numpy oracle, {threads} threads on {ncpu} host CPUs")


def h2d_probe(torch, nchan, ncols, pitch):
    """PCIe host->device rate for one pinned chunk: 1-D contiguous and 2-D strided copies."""
    dev = torch.device("cuda:0")
    src = torch.empty((nchan, pitch), dtype=torch.uint8).pin_memory()
    dst = torch.empty((nchan, ncols), dtype=torch.uint8, device=dev)
    flat = torch.empty(nchan * ncols, dtype=torch.uint8).pin_memory()
    dflat = torch.empty(nchan * ncols, dtype=torch.uint8, device=dev)
    out = {}
    for name, fn in (("h2d_1d_GBps", lambda: dflat.copy_(flat, non_blocking=True)),
                     ("h2d_2d_GBps", lambda: dst.copy_(src[:, :ncols], non_blocking=True))):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        out[name] = 5 * nchan * ncols / (time.perf_counter() - t) / 1e9
    return out


def stream_run(plan, src, nsamp, chunk, S, serial=False, sdma=False, staged=False, budget=16 << 30, cap=1 << 14,
               src_cols=None, reps=2, want_cands=False, min_piece_work=0):
    """One beam streamed through a pipeline: `nsamp` samples in chunks of `chunk`, read
    from `src` (uint8 [nchan, >= src_cols], pinned torch tensor or pageable numpy array).
    With src_cols < nsamp the source columns repeat: chunk k reads columns
    (k * chunk) mod src_cols. The first of `reps` passes warms copy engines and kernels;
    the last is reported. Returns wall time, union lengths of copy and kernel intervals
    (HIP events), H = overlap / copy union, E = max(copy union, kernel union) / span."""
    import torch

    from paper_2101_00941_amd import Pipeline
    src_cols = src_cols or nsamp
    pitch = src.stride(0) if hasattr(src, "stride") and callable(src.stride) else src.strides[0]
    out = None
    for _ in range(reps):
        pipe = Pipeline(nstreams=S, max_beams=1, max_chunk=chunk, cand_cap=cap, hbm_budget=budget, serial=serial,
                        timing=True, sdma_copy=sdma, staged=staged, min_piece_work=min_piece_work)
        b = pipe.add_beam(plan)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nk = 0
        for k, s0 in enumerate(range(0, nsamp, chunk)):
            n = min(chunk, nsamp - s0)
            c0 = s0 % src_cols
            assert c0 + n <= src_cols
            pipe.submit(b, src[:, c0:c0 + n], nsamp=n, pitch=pitch, tag=k, last=(s0 + n == nsamp))
            nk += 1
        ncand, cands, bad, over = 0, [], 0, 0
        for _ in range(nk):
            r = pipe.poll(timeout_us=60_000_000)
            assert r is not None, "pipeline stalled"
            bad += r["status"] not in (0, -5)
            over += r["status"] == -5
            ncand += r["n_true"]
            if want_cands:
                cands.extend((int(c["dm_idx"]), int(c["t"]), int(c["width"]), float(c["snr"])) for c in r["cand"])
        wall = time.perf_counter() - t0
        st = pipe.stats()
        pipe.close()
        assert bad == 0, "a chunk failed"
        out = dict(wall_ms=wall * 1e3, candidates=ncand, overflowed_chunks=over, **st)
        if want_cands:
            out["cand_list"] = sorted(cands, key=lambda c: (c[0], c[1]))
    out["hidden_frac"] = out["overlap_ms"] / out["copy_ms"] if out["copy_ms"] > 0 else None
    out["efficiency"] = max(out["copy_ms"], out["kernel_ms"]) / out["span_ms"] if out["span_ms"] > 0 else None
    return out


def _stream_rows(plan, host, nsamp, chunk, modes, budget, cap, src_cols=None, pageable=None, min_piece_work=0):
    # one untimed pass of every mode first: the first multi-stream pipelines of a process
    # ran slower than the same configuration later in it
    for mode, S, serial, sdma, is_pageable, staged in modes:
        stream_run(plan, pageable if is_pageable else host, nsamp, chunk, S, serial, sdma, staged, budget, cap,
                   src_cols, reps=1, min_piece_work=min_piece_work)
    rows = []
    for mode, S, serial, sdma, is_pageable, staged in modes:
        src = pageable if is_pageable else host
        r = stream_run(plan, src, nsamp, chunk, S, serial, sdma, staged, budget, cap, src_cols,
                       min_piece_work=min_piece_work)
        r.update(mode=mode, nstreams=S)
        r["dm_trial_samples_per_s"] = plan.info["ndm"] * (nsamp - plan.info["maxshift"]) / (r["wall_ms"] * 1e-3)
        rows.append(r)
        log(f"[bench] {mode} S={S}: {r['wall_ms']:.1f} ms wall, copy {r['copy_ms']:.1f} ms, kernels "
            f"{r['kernel_ms']:.1f} ms, overlap {r['overlap_ms']:.1f} ms, hidden {r['hidden_frac']}, "
            f"E {r['efficiency']}, {r['candidates']} candidates")
    plain = next(r["wall_ms"] for r in rows if r["mode"] == "plain")
    for r in rows:
        r["speedup_vs_plain"] = plain / r["wall_ms"]
    return rows


def streamed(a):
    """Streamed mode: a pinned host signal fed chunk by chunk through aa_stream_submit.
    Runs the paper's "before" mode (pageable input, no streams), the plain single-stream
    pipeline and then S = 1, 2, 4, 8 compute streams, and reports end-to-end rates,
    copy/kernel/overlap time and the hidden-transfer share."""
    import torch

    from paper_2101_00941_amd import Plan
    from synth.workloads import make_input, workload

    w = workload(a.workload)
    if a.ndm:
        w["dms"] = w["dms"][:a.ndm]
    chunk = w.get("chunk", 1 << 18)
    nsamp, nchan = w["nsamp"], w["nchan"]
    log(f"[bench] streamed {w['name']}: {nchan} x {nsamp}, chunks of {chunk}")
    host = torch.empty((nchan, nsamp), dtype=torch.uint8).pin_memory()
    make_input(w, out=host.numpy())
    torch.cuda.set_device(0)
    probe = h2d_probe(torch, nchan, chunk, nsamp)
    log(f"[bench] H2D probe {probe}")
    plan = Plan.from_workload(w)
    if a.variant != "auto":
        plan.set_variant(int(a.variant))
    budget = int(a.budget_gb * (1 << 30))
    # pageable copy of the same signal, for the paper's "before" mode (pageable input, no
    # streams) and for the pipeline's staged pageable input
    pageable = np.array(host.numpy(), copy=True)
    # (name, compute streams, serial, runtime copies, pageable input, staged)
    modes = ([("pageable-default", 1, True, False, True, False), ("plain", 1, True, False, False, False)]
             + [("streams", s, False, False, False, False) for s in a.streams]
             + [("streams-sdma", 2, False, True, False, False), ("pageable-staged", 4, False, False, True, True)])
    if a.only_streams:
        modes = [m for m in modes if m[0] in ("plain", "streams")]
    rows = _stream_rows(plan, host, nsamp, chunk, modes, budget, a.stream_cap, pageable=pageable,
                        min_piece_work=a.min_piece_work)
    return dict(workload=w["name"], chunk=chunk, ndm=plan.info["ndm"], nchan=nchan, nsamp=nsamp,
                dedisp_variant=plan.variant, h2d_probe=probe,
                hw_queues=os.environ.get("GPU_MAX_HW_QUEUES", "default"), runs=rows)


def streamed_compact(variant, budget_gb, cap, survey_host=None, resident_cands=None):
    """The streamed part of the default bench line.
    * streamed_128ch_8M: the 128-channel signal, 2^23 samples in 2^18 chunks (32 chunks).
    * survey_4096ch_streamed_16x: the survey plan over 16 chunks of 2^18 samples, read
      cyclically from the resident run's 2^20-sample pinned input. Its candidates over
      the starts that the first 2^20 samples determine must equal the resident run's."""
    import torch

    from paper_2101_00941_amd import Plan
    from synth.workloads import make_input, workload

    out = {}
    budget = int(budget_gb * (1 << 30))
    base = [("plain", 1, True, False, False, False)] + [("streams", s, False, False, False, False) for s in (1, 2, 4, 8)]
    w = workload("streamed_128ch_8M")
    host = torch.empty((w["nchan"], w["nsamp"]), dtype=torch.uint8).pin_memory()
    make_input(w, out=host.numpy())
    plan = Plan.from_workload(w)
    # the 128-channel plan is tuned on its own shape: one chunk plus the delay tail
    n_tune = min(w["nsamp"], w["chunk"] + plan.info["maxshift"])
    xt = torch.zeros((w["nchan"], (n_tune + 255) // 256 * 256), dtype=torch.uint8, device="cuda:0")
    xt[:, :n_tune].copy_(host[:, :n_tune])
    plan.autotune(xt, n_in=n_tune, reps=2)
    torch.cuda.synchronize()
    del xt
    log(f"[bench] streamed {w['name']} (dedispersion variant {plan.variant})")
    rows = _stream_rows(plan, host, w["nsamp"], w["chunk"], base, budget, cap)
    out[w["name"]] = _compact_rows(rows, chunks=w["nsamp"] // w["chunk"])
    out[w["name"]]["dedisp_variant"] = plan.variant
    del host
    if survey_host is not None:
        ws = workload("survey_4096ch_1M")
        plan = Plan.from_workload(ws)
        plan.set_variant(variant)
        chunk, nchunks = 1 << 18, 16
        log(f"[bench] streamed survey plan, {nchunks} chunks of {chunk}")
        modes = [("plain", 1, True, False, False, False)] + [("streams", s, False, False, False, False) for s in (2, 4)]
        # a strong pulse gives tens of thousands of candidates in one sub-chunk
        cap = max(cap, 1 << 18)
        rows = _stream_rows(plan, survey_host, nchunks * chunk, chunk, modes, budget, cap, src_cols=ws["nsamp"])
        res = _compact_rows(rows, chunks=nchunks)
        if resident_cands is not None:
            # starts below e = the first block-aligned start whose boxcars or right
            # neighbour reach past the first 2^20 samples are determined by them alone
            e = (ws["nsamp"] - plan.info["wmax"] - plan.info["maxshift"]) // plan.info["stat_block"] * plan.info["stat_block"]
            r = stream_run(plan, survey_host, 4 * chunk, chunk, 4, budget=budget, cap=cap, src_cols=ws["nsamp"], reps=1,
                           want_cands=True)
            got = [c for c in r["cand_list"] if c[1] < e]
            want = [c for c in resident_cands if c[1] < e]
            res["check"] = {"starts": e, "candidates": len(want), "overflowed_chunks": r["overflowed_chunks"],
                            "identical_to_resident": [c[:3] for c in got] == [c[:3] for c in want]
                            and all(abs(g[3] - h[3]) <= 1e-5 * max(1.0, abs(h[3])) for g, h in zip(got, want))}
            log(f"[bench] streamed survey vs resident over starts < {e}: {res['check']}")
        out["survey_4096ch_streamed_16x"] = res
    return out


def _compact_rows(rows, chunks):
    keep = ("wall_ms", "speedup_vs_plain", "hidden_frac", "efficiency", "copy_ms", "kernel_ms", "overlap_ms",
            "span_ms", "dm_trial_samples_per_s", "overflowed_chunks")
    out = {"chunks": chunks}
    for r in rows:
        key = r["mode"] if r["mode"] == "plain" else f"S{r['nstreams']}"
        out[key] = {k: (round(r[k], 4) if isinstance(r[k], float) else r[k]) for k in keep}
    return out


def serving(a):
    """Serving loop: 32 beams emit 2^17-sample chunks at Poisson times (0.5-2x real time,
    times `--rate-scale`). The continuous-batching pipeline (S compute streams, HBM-budget
    admission, device tails) is compared with the plain path (one stream, FIFO) on the
    same arrivals. Reports p50/p99 chunk latency (submit to result) and sustained rates."""
    import torch

    from paper_2101_00941_amd import Pipeline, Plan
    from synth.filterbank import Pulse, make_filterbank
    from synth.workloads import poisson_arrivals, serving_beams

    beams = serving_beams(nbeams=a.beams)
    chunk, nchan = beams[0]["chunk"], beams[0]["nchan"]
    torch.cuda.set_device(0)
    npool = 6
    log(f"[bench] serving: {len(beams)} beams, chunks of {chunk} x {nchan}, pool of {npool} chunks")
    pool = []
    for k in range(npool):
        h = torch.empty((nchan, chunk), dtype=torch.uint8).pin_memory()
        make_filterbank(nchan, chunk, 1450.0, 300.0 / 4096, 64e-6, [Pulse(300.0 + 100 * k, 60000.0, 8.0, 8.0)],
                        seed=100 + k, out=h.numpy())
        pool.append(h)
    plans = [Plan(nchan, 1 << 20, b["f_top"], b["foff"], b["tsamp"], b["dms"], b["widths"], b["threshold"],
                  b["stat_block"]) for b in beams]
    if a.variant != "auto":
        for p in plans:
            p.set_variant(int(a.variant))
    out = {}
    for scale in a.rate_scale:
        arrivals = poisson_arrivals(beams, a.serve_seconds, rate_scale=scale)
        for mode in ("continuous", "plain"):
            pipe = Pipeline(nstreams=1 if mode == "plain" else a.serve_streams, max_beams=len(beams),
                            max_chunk=chunk, cand_cap=a.stream_cap, hbm_budget=int(a.budget_gb * (1 << 30)),
                            serial=(mode == "plain"), result_slots=64)
            ids = [pipe.add_beam(p) for p in plans]
            nxt = [0] * len(beams)
            lat, work, done = [], 0, 0
            results = {}                     # tag -> (status, t range, candidate list)
            t0 = time.perf_counter()

            def drain(timeout):
                nonlocal work, done
                r = pipe.poll(timeout_us=timeout)
                while r is not None:
                    assert r["status"] in (0, -5), r
                    lat.append(r["latency_s"])
                    work += plans[r["beam"]].info["ndm"] * (r["t_end"] - r["t_begin"])
                    done += 1
                    results[r["tag"]] = (r["status"], r["t_begin"], r["t_end"], r["n_true"], r["cand"].tobytes())
                    r = pipe.poll(timeout_us=0)

            for i, (ta, b) in enumerate(arrivals):
                while True:
                    dt = ta - (time.perf_counter() - t0)
                    if dt <= 0:
                        break
                    drain(int(min(dt, 0.01) * 1e6))
                pipe.submit(ids[b], pool[(b + nxt[b]) % npool], nsamp=chunk, tag=i)
                nxt[b] += 1
            while done < len(arrivals):
                drain(1_000_000)
            wall = time.perf_counter() - t0
            st = pipe.stats()
            pipe.close()
            lat_ms = np.array(lat) * 1e3
            res = dict(chunks=len(arrivals), wall_s=wall, p50_ms=float(np.percentile(lat_ms, 50)),
                       p99_ms=float(np.percentile(lat_ms, 99)), mean_ms=float(lat_ms.mean()),
                       dm_trial_samples_per_s=work / wall, arena_peak_gb=st["arena_peak"] / 2**30)
            out[f"x{scale:g}_{mode}"] = res
            if mode == "continuous":
                first_results = results
            else:
                # every chunk's result in the mix equals the one-at-a-time (plain) result
                same = results.keys() == first_results.keys() and all(results[k] == first_results[k] for k in results)
                out[f"x{scale:g}_identical"] = bool(same)
                log(f"[bench] serving x{scale:g}: continuous and plain results identical: {same}")
            log(f"[bench] serving x{scale:g} {mode}: {len(arrivals)} chunks, p50 {res['p50_ms']:.1f} ms, "
                f"p99 {res['p99_ms']:.1f} ms, {res['dm_trial_samples_per_s']:.3e} DM-trial*samples/s, "
                f"arena peak {res['arena_peak_gb']:.1f} GB")
    return dict(workload="serving_32beams", chunk=chunk, nchan=nchan, beams=len(beams), dedisp_variant=plans[0].variant,
                seconds=a.serve_seconds, streams=a.serve_streams, hbm_budget_gb=a.budget_gb, results=out)


def batched(a):
    """Batched beams: 64 beams of uneven shape (nchan 1024/2048/4096, nsamp U[2^16, 2^20],
    500-3000 trials) generated on the device. The per-beam plain loop (aa_dedisperse +
    aa_single_pulse per beam) is compared with aa_batch_run (one persistent dedispersion
    launch per group, autotuned variant). Candidate lists must be identical."""
    import torch

    from paper_2101_00941_amd import Plan, batch_run, candidates_as_tuples, candidates_to_numpy
    from synth.filterbank_torch import make_filterbank_torch
    from synth.workloads import batched_beams

    torch.cuda.set_device(0)
    bs = batched_beams(nbeams=a.beams)
    t = time.perf_counter()
    beams = []
    for b in bs:
        x = make_filterbank_torch(b["nchan"], b["nsamp"], b["f_top"], b["foff"], b["tsamp"], b["pulses"],
                                  seed=b["seed"], device="cuda:0")
        plan = Plan(b["nchan"], b["nsamp"], b["f_top"], b["foff"], b["tsamp"], b["dms"], b["widths"],
                    b["threshold"], b["stat_block"])
        beams.append((plan, x, b["nsamp"]))
    torch.cuda.synchronize()
    in_gb = sum(x.numel() for _, x, _ in beams) / 1e9
    work_units = sum(p.info["ndm"] * p.info["n_dd"] for p, _, _ in beams)
    log(f"[bench] batched: {len(beams)} beams, {in_gb:.1f} GB input on device, made in {time.perf_counter() - t:.1f} s")
    cap = max(a.stream_cap, 1 << 20)   # a strong pulse gives tens of thousands of candidates per beam
    work = torch.empty(int(a.budget_gb * (1 << 30)), dtype=torch.uint8, device="cuda:0")
    # batch (autotuned once, then timed)
    cands, counts, info = batch_run(beams, variant=-1, work=work, cap=cap)
    torch.cuda.synchronize()
    t = time.perf_counter()
    cands, counts, info = batch_run(beams, variant=info["variant"], work=work, cap=cap)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    log(f"[bench] batch: {t_batch * 1e3:.1f} ms ({info})")
    # per-beam plain loop, same variant, same work buffer for the planes
    plain_counts, plain_cands = [], []
    t = time.perf_counter()
    for plan, x, n in beams:
        plan.set_variant(info["variant"])
        opitch = (plan.info["n_dd"] + 63) // 64 * 64
        dd = work[: plan.info["ndm"] * opitch * 4].view(torch.int32).view(plan.info["ndm"], opitch)
        plan.dedisperse(x, n_in=n, out=dd)
        c, cnt, _ = plan.single_pulse(dd, cap=cap)
        plain_counts.append(cnt)
        plain_cands.append(c)
    # both paths hand the candidate lists to the host inside their timed region
    plain_lists = [candidates_to_numpy(plain_cands[i], plain_counts[i], cap) for i in range(len(beams))]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    same = True
    for i in range(len(beams)):
        pc = candidates_as_tuples(plain_lists[i])
        same &= int(plain_counts[i].item()) == int(counts[i]) and pc == candidates_as_tuples(cands[i])
    log(f"[bench] plain loop: {t_plain * 1e3:.1f} ms; identical results: {same}")
    return dict(workload="batched_64beams", beams=len(beams), input_gb=in_gb, dm_trial_samples=work_units,
                overflowed_beams=int(sum(int(c) > cap for c in counts)),
                batch_ms=t_batch * 1e3, plain_ms=t_plain * 1e3,
                batch_dm_trial_samples_per_s=work_units / t_batch, plain_dm_trial_samples_per_s=work_units / t_plain,
                identical=bool(same), info=info)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="survey_4096ch_1M")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cap", type=int, default=1 << 20)
    ap.add_argument("--variant", default="auto",
                    help="dedispersion kernel variant, or 'auto' (resident and batched modes: the autotuner; "
                         "streamed and serving modes: the plan default)")
    ap.add_argument("--ndm", type=int, default=0, help="use only the first NDM trials (profiling runs)")
    ap.add_argument("--mode", default="resident", choices=["resident", "streamed", "serving", "batched", "decimated"])
    ap.add_argument("--streams", type=int, nargs="+", default=[1, 2, 4, 8], help="streamed mode: stream counts")
    ap.add_argument("--only-streams", action="store_true", help="streamed mode: plain and --streams runs only")
    ap.add_argument("--min-piece-work", type=int, default=0,
                    help="streamed mode: smallest sub-chunk (0: the library default 2^33, -1: always split)")
    ap.add_argument("--beams", type=int, default=32)
    ap.add_argument("--serve-seconds", type=float, default=20.0)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--rate-scale", type=float, nargs="+", default=[1.0, 4.0])
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--stream-cap", type=int, default=1 << 14)
    ap.add_argument("--hw-queues", type=int, default=0, help="GPU_MAX_HW_QUEUES for this process (<= 32)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference kernel for HBM counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="resident run only: leave out the compact streamed and serving runs")
    ap.add_argument("--serve-compact-s", type=float, default=6.0,
                    help="seconds of Poisson arrivals per serving run in the default bench line")
    a = ap.parse_args()
    if a.hw_queues:
        # HIP maps streams onto this many hardware queues; it must be set before HIP starts
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(a.hw_queues, 32))
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)

    if a.mode == "streamed":
        print(json.dumps(streamed(a)), flush=True)
        return
    if a.mode == "batched":
        if a.budget_gb == 16.0:
            a.budget_gb = 120.0
        if a.beams == 32:
            a.beams = 64
        print(json.dumps(batched(a)), flush=True)
        return
    if a.mode == "serving":
        if a.budget_gb == 16.0:
            a.budget_gb = 200.0
        print(json.dumps(serving(a)), flush=True)
        return
    if a.mode == "decimated":
        import torch

        from synth.workloads import make_input, workload
        w = workload("survey_4096ch_1M")
        pitch = (w["nsamp"] + 255) // 256 * 256
        x_host = torch.empty((w["nchan"], pitch), dtype=torch.uint8).pin_memory()
        make_input(w, pitch=pitch, out=x_host.numpy())
        torch.cuda.set_device(0)
        x = x_host.to("cuda:0")
        v = None if a.variant == "auto" else int(a.variant)
        print(json.dumps(decimated_run(w, x, v, torch.cuda.current_stream(), steps=a.steps)), flush=True)
        return

    import torch

    from paper_2101_00941_amd import Plan
    from synth.workloads import make_input, workload

    w = workload(a.workload)
    if a.ndm:
        w["dms"] = w["dms"][:a.ndm]
    log(f"[bench] generating {w['name']} ({w['nchan']} x {w['nsamp']} u8, {len(w['dms'])} DMs)")
    t = time.perf_counter()
    pitch = (w["nsamp"] + 255) // 256 * 256
    x_host = torch.empty((w["nchan"], pitch), dtype=torch.uint8).pin_memory()
    x_np = x_host.numpy()
    make_input(w, pitch=pitch, out=x_np)
    log(f"[bench] input ready in {time.perf_counter() - t:.1f} s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    plan = Plan.from_workload(w)
    info = plan.info
    ndm, n_dd, n_start, nchan = info["ndm"], info["n_dd"], info["n_start"], info["nchan"]
    x = x_host.to(dev, non_blocking=False)
    dd = torch.empty((ndm, info["out_pitch"]), dtype=torch.int32, device=dev)
    work = torch.empty(plan.work_bytes(n_start), dtype=torch.uint8, device=dev)
    cand = torch.empty(a.cap * 24, dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    h_cand = torch.empty(a.cap * 24, dtype=torch.uint8).pin_memory()
    h_count = torch.empty(1, dtype=torch.int32).pin_memory()
    stream = torch.cuda.current_stream()

    if a.variant == "auto":
        ms = plan.autotune(x, n_in=w["nsamp"], out=dd, reps=1)
        log(f"[bench] autotune ms per variant {['%.1f' % m for m in ms]} -> variant {plan.variant}")
    else:
        plan.set_variant(int(a.variant))

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.dedisperse(x, n_in=w["nsamp"], out=dd)
        if ev is not None:
            ev[1].record(stream)
        plan.single_pulse(dd, work=work, cand=cand, count=count, cap=a.cap)
        if ev is not None:
            ev[2].record(stream)
        h_count.copy_(count, non_blocking=True)
        h_cand.copy_(cand, non_blocking=True)

    if a.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for i in range(a.warmup):
        step()
        log(f"[bench] warmup {i + 1}/{a.warmup}")
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(evs[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_dedisp = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    ms_sps = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms_step = elapsed * 1000.0 / a.steps
    log(f"[bench] {a.steps} steps: {ms_step:.2f} ms/step (dedisp {ms_dedisp:.2f} ms, sps {ms_sps:.2f} ms), "
        f"{int(h_count.item())} candidates")

    adds = ndm * n_dd * nchan
    achieved = adds / (ms_dedisp * 1e-3) / 1e12
    value = ndm * n_dd / (ms_step * 1e-3)
    variants = Plan.variants()
    vinfo = variants[plan.variant]
    entry = TRAFFIC_BYTES.get((w["name"], plan.variant)) if not a.ndm else None
    traffic = entry[0] if entry and entry[1] == kernel_digest() else None
    if vinfo["layout"] in (4, 5, 6):
        # a contraction on the i8 matrix cores, priced against their dense peak; one op
        # per useful byte add (the one-hot weights are not counted)
        roofline = {"bound": "mfma", "dtype": "i8", "kernel": "dedisp_kernel (i8 matrix cores)",
                    "achieved": achieved, "peak": I8_MFMA_PEAK_TOPS, "unit": "TOP/s",
                    "frac": achieved / I8_MFMA_PEAK_TOPS, "traffic": traffic, "per_launch_ops": adds,
                    "ms_per_launch": ms_dedisp, "alu_peak": ALU_PEAK_TOPS, "alu_frac": achieved / ALU_PEAK_TOPS,
                    "hbm_frac": (ndm * n_dd * 4 + nchan * w["nsamp"]) / (ms_dedisp * 1e-3) / (HBM_PEAK_GBS * 1e9)}
    elif vinfo["layout"] == 7:
        roofline = quad_roofline(adds, ms_dedisp)
        roofline["traffic"] = traffic
    else:
        roofline = {"bound": "alu", "kernel": "dedisp_kernel", "achieved": achieved, "peak": ALU_PEAK_TOPS,
                    "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS, "traffic": traffic,
                    "per_launch_ops": adds, "ms_per_launch": ms_dedisp}
    res = {
        "metric": "DM-trial*samples/s per GPU (dedispersion + single-pulse search)",
        "value": value,
        "unit": "DM-trial*samples/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w["name"], "nchan": nchan, "nsamp": w["nsamp"], "ndm": ndm,
                   "dm_max": float(w["dms"][-1]), "widths": w["widths"], "stat_block": info["stat_block"],
                   "maxshift": info["maxshift"], "mode": "resident input, one stream",
                   "dedisp_variant": plan.variant},
        "roofline": roofline,
        "kernels_ms": {"dedisperse": ms_dedisp, "single_pulse": ms_sps},
        "candidates": int(h_count.item()),
    }
    if a.variant == "auto":
        # the best variant without matrix cores (shift-and-add: layouts 0-3 in packed
        # 16-bit adds, layout 7 with v_sad_u8 on staged channel quads), from the same
        # autotune pass (one timed launch each)
        sa = [(m, v) for v, m in enumerate(ms) if m > 0 and variants[v]["layout"] in (0, 1, 2, 3, 7)]
        if sa:
            m, v = min(sa)
            if variants[v]["layout"] == 7:
                res["shift_and_add"] = quad_roofline(adds, m)
            else:
                ach = adds / (m * 1e-3) / 1e12
                res["shift_and_add"] = {"bound": "alu", "achieved": ach, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                                        "frac": ach / ALU_PEAK_TOPS, "ms_per_launch": m}
            res["shift_and_add"].update(variant=v, value_if_used=ndm * n_dd / ((m + ms_sps) * 1e-3))
    if not a.no_extras and not a.ndm and w["name"] == "survey_4096ch_1M":
        res["decimated"] = decimated_run(w, x, None, stream)
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(w, x_np[:, :w["nsamp"]])
    if not a.no_extras and not a.ndm:
        n = min(int(h_count.item()), a.cap)
        raw = h_cand[: n * 24].numpy().view(_cand_dtype())
        resident = [(int(r["dm_idx"]), int(r["t"]), int(r["width"]), float(r["snr"])) for r in raw]
        del dd, work, x
        torch.cuda.empty_cache()
        res["streamed"] = streamed_compact(plan.variant, a.budget_gb, a.stream_cap, survey_host=x_host,
                                           resident_cands=resident)
        res["serving"] = serving_compact(a, plan.variant)
    print(json.dumps(res), flush=True)


SURVEY_RANGES = ([0, 512, 1024, 1536, 2048, 2432], [1, 2, 4, 8, 16, 32])


def quad_roofline(adds, ms):
    """Roofline of a quad shift-and-add launch: bound by LDS reads at one staged byte per
    byte-add (the algorithmic LDS bytes of an LDS-staged sum), with the v_sad_u8 VALU
    peak beside it."""
    gbs = adds / (ms * 1e-3) / 1e9
    return {"bound": "lds", "kernel": "dedisp_kernel (quad shift-and-add, v_sad_u8)", "achieved": gbs,
            "peak": LDS_PEAK_TBS * 1000.0, "unit": "GB/s", "frac": gbs / (LDS_PEAK_TBS * 1000.0),
            "per_launch_bytes": adds, "ms_per_launch": ms, "valu_peak_tops": SAD_PEAK_TOPS,
            "valu_frac": gbs / 1000.0 / SAD_PEAK_TOPS, "alu_frac": gbs / 1000.0 / ALU_PEAK_TOPS}


def decimated_run(w, x, variant, stream, steps=5):
    """Per-range time decimation on the resident survey input: the plan's six DM ranges
    (steps 1/16 .. 2) at factors 1, 2, 4, .. 32, one aa_range_run per step (decimation,
    dedispersion and search of every range). variant None autotunes each range on its
    own decimated input. Reports ms per run (HIP events on the launch stream), the
    input-sample rate and the adds it performs."""
    import ctypes as C

    import torch

    from paper_2101_00941_amd import RangePlan
    from paper_2101_00941_amd import _native as N
    first, factor = SURVEY_RANGES
    rp = RangePlan(w["nchan"], w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"],
                   first, factor, w["stat_block"])
    if variant is None:
        tuned = rp.autotune(x, n_in=w["nsamp"], reps=1)
        log(f"[bench] decimated ranges: autotuned variants {tuned}")
    else:
        rp.set_variant(variant)
        tuned = [variant] * len(first)
    cap = 1 << 20
    work = torch.empty(rp.work_bytes(w["nsamp"], cap), dtype=torch.uint8, device=x.device)
    cand = torch.empty(cap * 24, dtype=torch.uint8, device=x.device)
    count = torch.zeros(1, dtype=torch.int32, device=x.device)
    for _ in range(2):
        rp.run(x, n_in=w["nsamp"], cap=cap, work=work, cand=cand, count=count)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        rp.run(x, n_in=w["nsamp"], cap=cap, work=work, cand=cand, count=count)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ndm = len(w["dms"])
    from paper_2101_00941_amd import Plan
    n_dd_plain = Plan.from_workload(w, host_only=True).info["n_dd"]
    adds = 0   # algorithmic: trials x N_dd x channels of every range, N_dd at its resolution
    for r in range(len(first)):
        info = N.PlanInfo()
        N.check(N.lib().aa_plan_info(rp.range_plan(r)[0], C.byref(info)))
        adds += info.ndm * info.n_dd * info.nchan
    out = {"ranges_first": first, "factors": factor, "ms_per_run": ms, "candidates": int(count.item()),
           "input_samples_per_s": ndm * w["nsamp"] / (ms * 1e-3), "adds_per_run": adds,
           "adds_vs_plain": adds / (ndm * n_dd_plain * w["nchan"]), "dedisp_variants": tuned}
    log(f"[bench] decimated ranges: {ms:.2f} ms per run, {out['candidates']} candidates, "
        f"{out['adds_vs_plain']:.3f} of the plain adds")
    del work, cand, count, rp
    return out


def _cand_dtype():
    from paper_2101_00941_amd import _native
    return _native.CANDIDATE_DTYPE


def serving_compact(a, variant):
    """The serving part of the default bench line: serving_32beams for a.serve_compact_s
    seconds of arrivals at 1x and 4x real time, continuous batching against plain FIFO."""
    import copy
    b = copy.copy(a)
    b.serve_seconds, b.rate_scale, b.budget_gb, b.beams = a.serve_compact_s, [1.0, 4.0], 200.0, 32
    b.variant = str(variant)
    full = serving(b)
    out = {"beams": full["beams"], "seconds": full["seconds"], "streams": full["streams"],
           "hbm_budget_gb": full["hbm_budget_gb"], "dedisp_variant": full["dedisp_variant"]}
    for k, r in full["results"].items():
        if isinstance(r, bool):
            out[k] = r
            continue
        out[k] = {q: round(r[q], 4) for q in ("p50_ms", "p99_ms", "mean_ms", "dm_trial_samples_per_s")}
        out[k]["chunks"] = r["chunks"]
    return out


if __name__ == "__main__":
    main()
