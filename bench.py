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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, x, n_rows=9):
    """Time the oracle (as it is) on a bounded sample: the full time range for
    `n_rows` DM trials, i.e. three triples of neighbouring trials, so that the 3x3 peak
    test of each middle row has its neighbours. One process, numpy, one core."""
    import oracle
    ndm = len(w["dms"])
    centres = [ndm // 6, ndm // 2, (5 * ndm) // 6]
    rows = sorted({r for c in centres for r in (c - 1, c, c + 1)})[:n_rows]
    s = oracle.shift_table(w["dms"], w["nchan"], w["f_top"], w["foff"], w["tsamp"])
    sz = oracle.sizes(s, w["nsamp"], w["widths"], w["stat_block"])
    t0 = time.perf_counter()
    D = oracle.dedisperse_rows(x, s, rows, w["nsamp"], sz["maxshift"])
    for k in range(0, len(rows), 3):
        oracle.single_pulse(D[k:k + 3], 0, 0, sz["n_start"], sz["n_start"], w["widths"], w["threshold"],
                            w["stat_block"], row0=rows[k], ndm=ndm, report_rows=[rows[k + 1]])
    dt = time.perf_counter() - t0
    return dict(value=len(rows) * sz["n_dd"] / dt, unit="DM-trial*samples/s", cores=1, kind="oracle",
                sample=f"{len(rows)} DM trials ({', '.join(map(str, rows))}) x {sz['n_dd']} samples, "
                       f"dedispersion + single-pulse search, numpy, {dt:.1f} s")


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
    ndm = plan.info["ndm"]
    budget = int(a.budget_gb * (1 << 30))
    rows = []
    modes = [("plain", 1, False)] + [("streams", s, False) for s in (1, 2, 4, 8)] + [("streams-sdma", 2, True)]
    for mode, S, sdma in modes:
        best = None
        for rep in range(2):   # first pass warms up copy engines and kernels
            pipe = Pipeline(nstreams=S, max_beams=1, max_chunk=chunk, cand_cap=a.stream_cap, hbm_budget=budget,
                            serial=(mode == "plain"), timing=True, sdma_copy=sdma)
            b = pipe.add_beam(plan)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nk = 0
            for k, s0 in enumerate(range(0, nsamp, chunk)):
                n = min(chunk, nsamp - s0)
                pipe.submit(b, host[:, s0:s0 + n], nsamp=n, pitch=nsamp, tag=k, last=(s0 + n == nsamp))
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
    plain = rows[0]["wall_ms"]
    for r in rows:
        r["speedup_vs_plain"] = plain / r["wall_ms"]
    return dict(workload=w["name"], chunk=chunk, ndm=ndm, nchan=nchan, nsamp=nsamp, h2d_probe=probe,
                hw_queues=os.environ.get("GPU_MAX_HW_QUEUES", "default"), runs=rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="survey_4096ch_1M")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cap", type=int, default=1 << 20)
    ap.add_argument("--variant", default="auto", help="dedispersion kernel variant, or 'auto' (autotuner)")
    ap.add_argument("--ndm", type=int, default=0, help="use only the first NDM trials (profiling runs)")
    ap.add_argument("--mode", default="resident", choices=["resident", "streamed"])
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--stream-cap", type=int, default=1 << 14)
    ap.add_argument("--hw-queues", type=int, default=0, help="GPU_MAX_HW_QUEUES for this process (<= 32)")
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
        "roofline": {"bound": "alu", "kernel": "dedisp_kernel", "achieved": achieved, "peak": ALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS, "traffic": None,
                     "per_launch_ops": adds, "ms_per_launch": ms_dedisp},
        "kernels_ms": {"dedisperse": ms_dedisp, "single_pulse": ms_sps},
        "candidates": int(h_count.item()),
    }
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(w, x_np[:, :w["nsamp"]])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
