"""Benchmark: brute-force dedispersion + single-pulse search on one MI355X.

Default workload: survey_4096ch_1M. That is 4096 channels x 2^20 uint8 samples,
3000 DM trials of the doubling-step plan (0..1998), boxcars 1..256 and threshold 6.
The input is resident in HBM. One step is the whole hot path over that input:
aa_dedisperse (all trials, every sample), then aa_single_pulse (block statistics,
boxcar S/N, 3x3 peaks and ordered candidates), then the asynchronous copy of the
candidate count and list to pinned host memory.

Prints ONE JSON line with the metric, a roofline object for the dominant kernel
(dedispersion, measured with HIP events on its own stream), and the CPU oracle
timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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
# Dense int8 matrix-core peak (v_mfma_i32_*_i8), TOP/s.
I8_MFMA_PEAK_TOPS = 5000.0
# HBM bytes per launch of the dedispersion kernel (FETCH_SIZE x 2.000 + WRITE_SIZE x
# 1.000 per dispatch, scaled by a 1 GiB copy), from the counter runs summarised in
# profiles/dedisp_*_survey_4096ch_1M.md. Keyed by (workload, variant); valid only for
# the kernel code those counters were taken on.
TRAFFIC_BYTES = {
    ("survey_4096ch_1M", 12): 175.5e9 + 12.15e9,
    ("survey_4096ch_1M", 17): 279.1e9 + 12.15e9,
    ("survey_4096ch_1M", 20): 202.0e9 + 12.15e9,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


_CPU = {}


def _cpu_triple(centre):
    """Oracle on one triple of neighbouring trials: dedisperse rows centre-1..centre+1 over
    the full time range, then search the centre row (it needs both neighbours)."""
    import oracle
    w, x, s, sz = _CPU["w"], _CPU["x"], _CPU["s"], _CPU["sz"]
    rows = [centre - 1, centre, centre + 1]
    t0 = time.perf_counter()
    D = oracle.dedisperse_rows(x, s, rows, w["nsamp"], sz["maxshift"])
    oracle.single_pulse(D, 0, 0, sz["n_start"], sz["n_start"], w["widths"], w["threshold"], w["stat_block"],
                        row0=rows[0], ndm=len(w["dms"]), report_rows=[centre])
    return time.perf_counter() - t0


def cpu_baseline(w, x, n_centres=10):
    """Time the oracle (as it is) on a bounded sample: `n_centres` DM trials spread evenly
    over the plan (every ndm / n_centres-th), each searched over the full time range with
    its two neighbour rows dedispersed as well. The triples run in a thread pool over the
    host's cores (at most 16 threads); numpy is single-threaded here. value counts only the
    searched centre rows. Threads, not processes: the oracle's large numpy operations
    release the GIL, and no process forks after the GPU is initialised."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    ndm = len(w["dms"])
    step = ndm // n_centres
    centres = [min(max(1, step // 2 + k * step), ndm - 2) for k in range(n_centres)]
    s = oracle.shift_table(w["dms"], w["nchan"], w["f_top"], w["foff"], w["tsamp"])
    sz = oracle.sizes(s, w["nsamp"], w["widths"], w["stat_block"])
    _CPU.update(w=w, x=x, s=s, sz=sz)
    cores = max(1, min(16, os.cpu_count() or 1, n_centres))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as pool:
        per = list(pool.map(_cpu_triple, centres))
    wall = time.perf_counter() - t0
    cpu = float(sum(per))
    return dict(value=n_centres * sz["n_dd"] / wall, unit="DM-trial*samples/s", cores=cores, kind="oracle",
                per_triple_value=n_centres * sz["n_dd"] / cpu,
                sample=f"{n_centres} DM trials (every {step}th: {centres[0]}..{centres[-1]}), each with its 2 neighbour "
                       f"rows dedispersed, x {sz['n_dd']} samples, dedispersion + single-pulse search, numpy, "
                       f"{cores} threads, {wall:.1f} s wall, {cpu:.1f} s summed over the triples")


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


def streamed(a):
    """Streamed mode: a pinned host signal fed chunk by chunk through aa_stream_submit.
    Runs the plain single-stream pipeline and then S = 1, 2, 4, 8 compute streams, and
    reports end-to-end rates, copy/kernel/overlap time and the hidden-transfer share."""
    import torch

    from paper_2101_00941_amd import Pipeline, Plan
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
    ndm = plan.info["ndm"]
    budget = int(a.budget_gb * (1 << 30))
    rows = []
    # pageable copy of the same signal, for the paper's "before" mode (pageable input, no
    # streams) and for the pipeline's staged pageable input
    pageable = np.array(host.numpy(), copy=True)
    # (name, compute streams, serial, runtime copies, pageable input, staged)
    modes = ([("pageable-default", 1, True, False, True, False), ("plain", 1, True, False, False, False)]
             + [("streams", s, False, False, False, False) for s in (1, 2, 4, 8)]
             + [("streams-sdma", 2, False, True, False, False), ("pageable-staged", 4, False, False, True, True)])
    for mode, S, serial, sdma, is_pageable, staged in modes:
        best = None
        src_arr = pageable if is_pageable else host
        for rep in range(2):   # first pass warms up copy engines and kernels
            pipe = Pipeline(nstreams=S, max_beams=1, max_chunk=chunk, cand_cap=a.stream_cap, hbm_budget=budget,
                            serial=serial, timing=True, sdma_copy=sdma, staged=staged)
            b = pipe.add_beam(plan)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nk = 0
            for k, s0 in enumerate(range(0, nsamp, chunk)):
                n = min(chunk, nsamp - s0)
                pipe.submit(b, src_arr[:, s0:s0 + n], nsamp=n, pitch=nsamp, tag=k, last=(s0 + n == nsamp))
                nk += 1
            ncand = 0
            for _ in range(nk):
                r = pipe.poll(timeout_us=60_000_000)
                assert r is not None and r["status"] in (0, -5), r
                ncand += r["n_true"]
            wall = time.perf_counter() - t0
            st = pipe.stats()
            pipe.close()
            best = dict(mode=mode, nstreams=S, wall_ms=wall * 1e3, candidates=ncand, **st)
        T = plan.info["n_start"]
        best["dm_trial_samples_per_s"] = ndm * (nsamp - plan.info["maxshift"]) / (best["wall_ms"] * 1e-3)
        best["samples_per_s"] = nsamp / (best["wall_ms"] * 1e-3)
        best["hidden_frac"] = best["overlap_ms"] / best["copy_ms"] if best["copy_ms"] > 0 else None
        best["efficiency"] = (max(best["copy_sum_ms"], best["kernel_sum_ms"]) / best["span_ms"]
                              if best["span_ms"] > 0 else None)
        rows.append(best)
        log(f"[bench] {mode} S={S}: {best['wall_ms']:.1f} ms wall, copy {best['copy_ms']:.1f} ms, "
            f"kernels {best['kernel_ms']:.1f} ms, overlap {best['overlap_ms']:.1f} ms, "
            f"hidden {best['hidden_frac']}, {best['candidates']} candidates")
    plain = next(r["wall_ms"] for r in rows if r["mode"] == "plain")
    for r in rows:
        r["speedup_vs_plain"] = plain / r["wall_ms"]
    return dict(workload=w["name"], chunk=chunk, ndm=ndm, nchan=nchan, nsamp=nsamp, dedisp_variant=plan.variant,
                h2d_probe=probe,
                hw_queues=os.environ.get("GPU_MAX_HW_QUEUES", "default"), runs=rows)


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
            t0 = time.perf_counter()

            def drain(timeout):
                nonlocal work, done
                r = pipe.poll(timeout_us=timeout)
                while r is not None:
                    assert r["status"] in (0, -5), r
                    lat.append(r["latency_s"])
                    work += plans[r["beam"]].info["ndm"] * (r["t_end"] - r["t_begin"])
                    done += 1
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
    cap = a.stream_cap
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
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    same = True
    for i in range(len(beams)):
        pc = candidates_as_tuples(candidates_to_numpy(plain_cands[i], plain_counts[i], cap))
        same &= int(plain_counts[i].item()) == int(counts[i]) and pc == candidates_as_tuples(cands[i])
    log(f"[bench] plain loop: {t_plain * 1e3:.1f} ms; identical results: {same}")
    return dict(workload="batched_64beams", beams=len(beams), input_gb=in_gb, dm_trial_samples=work_units,
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
    ap.add_argument("--mode", default="resident", choices=["resident", "streamed", "serving", "batched"])
    ap.add_argument("--beams", type=int, default=32)
    ap.add_argument("--serve-seconds", type=float, default=20.0)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--rate-scale", type=float, nargs="+", default=[1.0, 4.0])
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--stream-cap", type=int, default=1 << 14)
    ap.add_argument("--hw-queues", type=int, default=0, help="GPU_MAX_HW_QUEUES for this process (<= 32)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference kernel for HBM counters)")
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
    vinfo = Plan.variants()[plan.variant]
    traffic = TRAFFIC_BYTES.get((w["name"], plan.variant)) if not a.ndm else None
    if vinfo["layout"] in (4, 5, 6):
        # a contraction on the i8 matrix cores, priced against their dense peak; one op
        # per useful byte add (the one-hot weights are not counted)
        roofline = {"bound": "mfma", "dtype": "i8", "kernel": "dedisp_kernel (i8 matrix cores)",
                    "achieved": achieved, "peak": I8_MFMA_PEAK_TOPS, "unit": "TOP/s",
                    "frac": achieved / I8_MFMA_PEAK_TOPS, "traffic": traffic, "per_launch_ops": adds,
                    "ms_per_launch": ms_dedisp, "alu_peak": ALU_PEAK_TOPS, "alu_frac": achieved / ALU_PEAK_TOPS}
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
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(w, x_np[:, :w["nsamp"]])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
