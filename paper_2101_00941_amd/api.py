"""Python binding with the C ABI's names. It marshals arguments only.

PyTorch supplies device memory and streams: torch.cuda tensors are passed by
pointer, and the current torch stream, or the one given, is passed as a
hipStream_t. Every step of the computation runs in the HIP library.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Plan:
    """aa_plan: float64 shift table, sizes and the one-time device upload."""

    def __init__(self, nchan, nsamp, f_top, foff, tsamp, dms, widths, threshold, stat_block=0, host_only=False,
                 clip_sigma=0.0, clip_iters=0, boxcar_full_width=0):
        L = N.lib()
        self._dm = np.ascontiguousarray(np.asarray(dms, dtype=np.float64))
        self._w = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
        d = N.PlanDesc()
        d.nchan = int(nchan)
        d.nsamp = int(nsamp)
        d.f_top_mhz = float(f_top)
        d.foff_mhz = float(foff)
        d.tsamp_s = float(tsamp)
        d.dm = self._dm.ctypes.data_as(C.POINTER(C.c_double))
        d.ndm = len(self._dm)
        d.widths = self._w.ctypes.data_as(C.POINTER(C.c_int32))
        d.nwidths = len(self._w)
        d.snr_threshold = float(threshold)
        d.stat_block = int(stat_block)
        d.flags = N.AA_PLAN_HOST_ONLY if host_only else 0
        d.clip_sigma = float(clip_sigma)
        d.clip_iters = int(clip_iters)
        d.boxcar_full_width = int(boxcar_full_width)
        h = C.c_void_p()
        N.check(L.aa_plan(C.byref(d), C.byref(h)))
        self._h = h
        inf = N.PlanInfo()
        N.check(L.aa_plan_info(h, C.byref(inf)))
        self.info = {k: getattr(inf, k) for k, _ in N.PlanInfo._fields_}
        self.threshold = float(np.float32(threshold))
        self.widths = [int(x) for x in self._w]
        self.dms = self._dm.copy()

    @classmethod
    def from_workload(cls, w, **kw):
        return cls(w["nchan"], w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"],
                   w["threshold"], w.get("stat_block", 0), **kw)

    @property
    def handle(self):
        return self._h

    def __getattr__(self, k):
        info = self.__dict__.get("info")
        if info is not None and k in info:
            return info[k]
        raise AttributeError(k)

    def close(self):
        if getattr(self, "_h", None):
            N.lib().aa_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shifts(self) -> np.ndarray:
        out = np.empty((self.info["ndm"], self.info["nchan"]), dtype=np.int32)
        N.check(N.lib().aa_plan_shifts(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    # ---- compute -------------------------------------------------------------
    def dedisperse(self, x, n_in=None, out=None, stream=None):
        """aa_dedisperse. x: uint8 CUDA tensor [nchan, in_pitch]. Returns int32 [ndm, out_pitch]."""
        import torch
        if x.dtype != torch.uint8 or not x.is_cuda or x.dim() != 2 or not x.is_contiguous():
            raise ValueError("x must be a contiguous uint8 CUDA tensor [nchan, pitch]")
        if x.shape[0] < self.info["nchan"]:
            raise ValueError("x has fewer rows than the plan has channels")
        n_in = x.shape[1] if n_in is None else int(n_in)
        if n_in > x.shape[1]:
            raise ValueError("n_in exceeds the row length of x")
        n_out = n_in - self.info["maxshift"]
        if out is None:
            pitch = (max(n_out, 1) + 63) // 64 * 64
            out = torch.empty((self.info["ndm"], pitch), dtype=torch.int32, device=x.device)
        elif (out.dtype != torch.int32 or out.dim() != 2 or out.shape[0] < self.info["ndm"]
              or out.shape[1] < n_out or out.stride(1) != 1):
            raise ValueError("out must be int32 [ndm, >= n_out] with unit column stride")
        N.check(N.lib().aa_dedisperse(self._h, _ptr(x), x.stride(0), n_in, _ptr(out), out.stride(0),
                                      _stream_handle(stream)))
        return out

    @staticmethod
    def variants():
        L = N.lib()
        out = []
        for v in range(L.aa_variant_count()):
            vi = N.VariantInfo()
            N.check(L.aa_variant_info(v, C.byref(vi)))
            out.append({k: getattr(vi, k) for k, _ in N.VariantInfo._fields_})
        return out

    @property
    def variant(self):
        v = C.c_int32()
        N.check(N.lib().aa_plan_get_variant(self._h, C.byref(v)))
        return v.value

    def set_variant(self, v):
        N.check(N.lib().aa_plan_set_variant(self._h, int(v)))

    def autotune(self, x, n_in=None, out=None, reps=2, stream=None):
        """aa_autotune on the caller's buffers. Returns the per-variant mean ms (-1: from cache)."""
        import torch
        n_in = x.shape[1] if n_in is None else int(n_in)
        n_out = n_in - self.info["maxshift"]
        if out is None:
            out = torch.empty((self.info["ndm"], (n_out + 63) // 64 * 64), dtype=torch.int32, device=x.device)
        nv = N.lib().aa_variant_count()
        ms = (C.c_float * nv)()
        N.check(N.lib().aa_autotune(self._h, _ptr(x), x.stride(0), n_in, _ptr(out), out.stride(0), int(reps),
                                    _stream_handle(stream), ms))
        return [float(v) for v in ms]

    def work_bytes(self, n_starts):
        v = C.c_size_t()
        N.check(N.lib().aa_single_pulse_work_bytes(self._h, int(n_starts), C.byref(v)))
        return v.value

    def single_pulse(self, dd, dd_t0=0, dd_n=None, t_begin=0, t_end=None, t_total=None, cap=1 << 16,
                     want_best=False, work=None, cand=None, count=None, stream=None):
        """aa_single_pulse. Returns (cand uint8 [cap*24] tensor, count int32 [1] tensor, best or None).

        Use `candidates_to_numpy(cand, count)` after the stream has finished.
        """
        import torch
        if dd.dtype != torch.int32 or not dd.is_cuda or dd.dim() != 2:
            raise ValueError("dd must be an int32 CUDA tensor [ndm, pitch]")
        if dd.shape[0] < self.info["ndm"] or dd.stride(1) != 1:
            raise ValueError("dd must have ndm rows and unit column stride")
        dd_n = min(self.info["n_dd"] - dd_t0, dd.shape[1]) if dd_n is None else int(dd_n)
        if dd_n > dd.shape[1]:
            raise ValueError("dd_n exceeds the row length of dd")
        t_end = self.info["n_start"] if t_end is None else int(t_end)
        t_total = self.info["n_start"] if t_total is None else int(t_total)
        n = t_end - t_begin
        wb = self.work_bytes(n)
        dev = dd.device
        if work is None or work.numel() < wb:
            work = torch.empty(wb, dtype=torch.uint8, device=dev)
        if cand is None:
            cand = torch.empty(max(cap, 1) * 24, dtype=torch.uint8, device=dev)
        elif cand.numel() < cap * 24 or cand.dtype != torch.uint8:
            raise ValueError("cand must be a uint8 buffer of at least cap * 24 bytes")
        if count is None:
            count = torch.zeros(1, dtype=torch.int32, device=dev)
        best = None
        if want_best:
            best = torch.empty((self.info["ndm"], (n + 63) // 64 * 64), dtype=torch.float32, device=dev)
        N.check(N.lib().aa_single_pulse(self._h, _ptr(dd), dd.stride(0), int(dd_t0), dd_n, int(t_begin), t_end,
                                        t_total, _ptr(work), work.numel(), _ptr(cand), int(cap), _ptr(count),
                                        _ptr(best) if best is not None else None,
                                        best.stride(0) if best is not None else 0, _stream_handle(stream)))
        return cand, count, best

    def single_pulse_noalloc(self, dd, cand, count, dd_t0=0, dd_n=None, t_begin=0, t_end=None, t_total=None,
                             cap=None, best=None, stream=None):
        """aa_single_pulse_noalloc: the search with the library's fixed scratch (no work
        buffer, nothing allocated by the call). cand, count (and best) are the caller's."""
        import torch
        if dd.dtype != torch.int32 or not dd.is_cuda or dd.dim() != 2 or dd.stride(1) != 1:
            raise ValueError("dd must be an int32 CUDA tensor [ndm, pitch] with unit column stride")
        dd_n = min(self.info["n_dd"] - dd_t0, dd.shape[1]) if dd_n is None else int(dd_n)
        t_end = self.info["n_start"] if t_end is None else int(t_end)
        t_total = self.info["n_start"] if t_total is None else int(t_total)
        cap = cand.numel() // 24 if cap is None else int(cap)
        if cand.dtype != torch.uint8 or cand.numel() < cap * 24:
            raise ValueError("cand must be a uint8 buffer of at least cap * 24 bytes")
        N.check(N.lib().aa_single_pulse_noalloc(self._h, _ptr(dd), dd.stride(0), int(dd_t0), dd_n, int(t_begin), t_end,
                                                t_total, _ptr(cand), cap, _ptr(count),
                                                _ptr(best) if best is not None else None,
                                                best.stride(0) if best is not None else 0, _stream_handle(stream)))
        return cand, count, best


def decimate2(x, n_in=None, out=None, stream=None):
    """aa_decimate2: one rounding-average halving of every row of a uint8 CUDA tensor."""
    import torch
    n_in = x.shape[1] if n_in is None else int(n_in)
    if out is None:
        out = torch.empty((x.shape[0], (n_in // 2 + 255) // 256 * 256), dtype=torch.uint8, device=x.device)
    N.check(N.lib().aa_decimate2(_ptr(x), x.stride(0), n_in, x.shape[0], _ptr(out), out.stride(0),
                                 _stream_handle(stream)))
    return out


class RangePlan:
    """aa_range_plan: per-range time decimation over one plan description."""

    def __init__(self, nchan, nsamp, f_top, foff, tsamp, dms, widths, threshold, first, factor, stat_block=0,
                 clip_sigma=0.0, clip_iters=0, boxcar_full_width=0):
        self._dm = np.ascontiguousarray(np.asarray(dms, dtype=np.float64))
        self._w = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
        d = N.PlanDesc()
        d.nchan, d.nsamp = int(nchan), int(nsamp)
        d.f_top_mhz, d.foff_mhz, d.tsamp_s = float(f_top), float(foff), float(tsamp)
        d.dm = self._dm.ctypes.data_as(C.POINTER(C.c_double))
        d.ndm = len(self._dm)
        d.widths = self._w.ctypes.data_as(C.POINTER(C.c_int32))
        d.nwidths = len(self._w)
        d.snr_threshold = float(threshold)
        d.stat_block = int(stat_block)
        d.flags = 0
        d.clip_sigma = float(clip_sigma)
        d.clip_iters = int(clip_iters)
        d.boxcar_full_width = int(boxcar_full_width)
        fa = (C.c_int32 * len(first))(*[int(v) for v in first])
        fb = (C.c_int32 * len(factor))(*[int(v) for v in factor])
        h = C.c_void_p()
        N.check(N.lib().aa_range_plan(C.byref(d), fa, fb, len(first), C.byref(h)))
        self._h = h
        self.nchan = int(nchan)
        self.first = [int(v) for v in first]
        self.factor = [int(v) for v in factor]

    def range_plan(self, r):
        """(plan handle, first trial, factor) of range r; the handle stays owned here."""
        p, a, f = C.c_void_p(), C.c_int32(), C.c_int32()
        N.check(N.lib().aa_range_plan_get(self._h, int(r), C.byref(p), C.byref(a), C.byref(f)))
        return p, a.value, f.value

    def set_variant(self, v):
        for r in range(len(self.first)):
            N.check(N.lib().aa_plan_set_variant(self.range_plan(r)[0], int(v)))

    def work_bytes(self, n_in, cap):
        v = C.c_size_t()
        N.check(N.lib().aa_range_work_bytes(self._h, int(n_in), int(cap), C.byref(v)))
        return v.value

    def autotune(self, x, n_in=None, reps=1, work=None, stream=None):
        """aa_range_autotune: each range's fastest variant on its own decimated input.
        Returns the chosen variant per range."""
        import torch
        n_in = x.shape[1] if n_in is None else int(n_in)
        wb = self.work_bytes(n_in, 0)
        if work is None or work.numel() < wb:
            work = torch.empty(wb, dtype=torch.uint8, device=x.device)
        nv = N.lib().aa_variant_count()
        ms = (C.c_float * (nv * len(self.first)))()
        N.check(N.lib().aa_range_autotune(self._h, _ptr(x), x.stride(0), n_in, _ptr(work), work.numel(), int(reps),
                                          _stream_handle(stream), ms))
        self.tune_ms = [[float(ms[r * nv + v]) for v in range(nv)] for r in range(len(self.first))]
        out = []
        for r in range(len(self.first)):
            v = C.c_int32()
            N.check(N.lib().aa_plan_get_variant(self.range_plan(r)[0], C.byref(v)))
            out.append(v.value)
        return out

    def run(self, x, n_in=None, cap=1 << 16, work=None, cand=None, count=None, stream=None):
        """aa_range_run. Returns (cand uint8 [cap*24] tensor, count int32 [1] tensor)."""
        import torch
        n_in = x.shape[1] if n_in is None else int(n_in)
        wb = self.work_bytes(n_in, cap)
        if work is None or work.numel() < wb:
            work = torch.empty(wb, dtype=torch.uint8, device=x.device)
        if cand is None:
            cand = torch.empty(max(cap, 1) * 24, dtype=torch.uint8, device=x.device)
        if count is None:
            count = torch.zeros(1, dtype=torch.int32, device=x.device)
        N.check(N.lib().aa_range_run(self._h, _ptr(x), x.stride(0), n_in, _ptr(work), work.numel(), _ptr(cand),
                                     int(cap), _ptr(count), _stream_handle(stream)))
        return cand, count

    def close(self):
        if getattr(self, "_h", None):
            N.lib().aa_range_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cluster(cand, dm_radius, t_radius):
    """aa_cluster over a host structured candidate array (CANDIDATE_DTYPE). Returns a
    structured array of clusters (peak, members, dm_lo, dm_hi, t_lo, t_hi)."""
    cand = np.ascontiguousarray(cand, dtype=N.CANDIDATE_DTYPE)
    n = len(cand)
    cap = max(n, 1)
    out = np.zeros(cap, dtype=N.CLUSTER_DTYPE)
    m = C.c_int64()
    N.check(N.lib().aa_cluster(cand.ctypes.data_as(C.c_void_p) if n else None, n, int(dm_radius), int(t_radius),
                               out.ctypes.data_as(C.c_void_p), cap, C.byref(m)))
    return out[: m.value].copy()


def candidates_to_numpy(cand, count, cap=None):
    """Copy a candidate buffer to the host as a structured array (dm_idx, width, t, snr, beam)."""
    n = int(count.item()) if hasattr(count, "item") else int(count)
    cap = cand.numel() // 24 if cap is None else cap
    n = min(n, cap)
    raw = cand[: n * 24].cpu().numpy()
    return raw.view(N.CANDIDATE_DTYPE).copy()


def candidates_as_tuples(arr):
    return [(int(r["dm_idx"]), int(r["t"]), int(r["width"]), float(r["snr"])) for r in arr]


class Pipeline:
    """aa_pipeline_*: streamed chunks over HIP streams with per-beam device tails.

    submit() takes host memory as a torch uint8 tensor or a numpy array. Pinned memory
    (torch pin_memory) takes the fast copy paths; pageable memory is staged by the
    runtime, or by the pipeline's pinned bounce buffers when staged=True. The memory
    must stay untouched until poll() has returned the chunk's tag.
    """

    def __init__(self, nstreams=4, max_beams=1, max_chunk=1 << 18, cand_cap=1 << 14, result_slots=0,
                 hbm_budget=8 << 30, serial=False, timing=False, sdma_copy=False, staged=False, min_piece_work=0):
        o = N.PipelineOpts()
        o.nstreams, o.max_beams, o.max_chunk = int(nstreams), int(max_beams), int(max_chunk)
        o.cand_cap, o.result_slots, o.hbm_budget = int(cand_cap), int(result_slots), int(hbm_budget)
        o.min_piece_work = int(min_piece_work)
        o.flags = ((N.AA_PIPE_SERIAL if serial else 0) | (N.AA_PIPE_TIMING if timing else 0)
                   | (N.AA_PIPE_SDMA_COPY if sdma_copy else 0) | (N.AA_PIPE_STAGED if staged else 0))
        h = C.c_void_p()
        N.check(N.lib().aa_pipeline_create(C.byref(o), C.byref(h)))
        self._h = h
        self._keep = {}
        self.plans = []

    def add_beam(self, plan, t_resume=None):
        """aa_pipeline_add_beam, or aa_pipeline_add_beam_at when t_resume is given."""
        b = C.c_int32()
        if t_resume is None:
            N.check(N.lib().aa_pipeline_add_beam(self._h, plan.handle, C.byref(b)))
        else:
            N.check(N.lib().aa_pipeline_add_beam_at(self._h, plan.handle, int(t_resume), C.byref(b)))
        self.plans.append(plan)
        return b.value

    def submit(self, beam, host, nsamp=None, tag=0, last=False, pitch=None):
        """host: uint8 [nchan, pitch], a torch tensor or a numpy array. Pinned memory takes
        the fast copy paths; pageable memory is staged by the runtime, or by the pipeline's
        bounce buffers when it was created with staged=True."""
        if hasattr(host, "data_ptr"):
            ptr, rows, cols, rp = host.data_ptr(), host.shape[0], host.shape[1], host.stride(0)
        else:
            ptr, rows, cols, rp = host.ctypes.data, host.shape[0], host.shape[1], host.strides[0]
        nsamp = cols if nsamp is None else int(nsamp)
        N.check(N.lib().aa_stream_submit(self._h, int(beam), C.c_void_p(ptr), nsamp, int(pitch or rp),
                                         int(tag), N.AA_SUBMIT_LAST if last else 0))
        self._keep[int(tag)] = host

    def poll(self, timeout_us=-1):
        """Returns None (nothing finished in time) or a dict with a structured candidate array."""
        r = N.Result()
        rc = N.check(N.lib().aa_poll(self._h, C.byref(r), int(timeout_us)))
        if rc == N.AA_EAGAIN:
            return None
        n = int(r.n)
        if n:
            buf = (C.c_uint8 * (n * 24)).from_address(r.cand)
            cand = np.frombuffer(buf, dtype=N.CANDIDATE_DTYPE, count=n).copy()
        else:
            cand = np.zeros(0, dtype=N.CANDIDATE_DTYPE)
        N.check(N.lib().aa_release(self._h, r.tag))
        self._keep.pop(int(r.tag), None)
        return dict(tag=int(r.tag), beam=int(r.beam), status=int(r.status), t_begin=int(r.t_begin),
                    t_end=int(r.t_end), n_true=int(r.n_true), cand=cand, latency_s=float(r.latency_s),
                    queue_s=float(r.queue_s))

    def stats(self):
        st = N.PipelineStats()
        N.check(N.lib().aa_pipeline_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in N.PipelineStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            N.check(N.lib().aa_pipeline_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_run(beams, variant=-1, work=None, work_bytes=None, cap=1 << 16, static=False, stream=None):
    """aa_batch_run. beams: list of (Plan, uint8 CUDA tensor [nchan, pitch], n_in).
    Returns (list of per-beam structured candidate arrays, true counts, info dict)."""
    import torch
    n = len(beams)
    arr = (N.BatchBeam * n)()
    for i, (plan, x, n_in) in enumerate(beams):
        if x.dtype != torch.uint8 or not x.is_cuda or x.shape[0] < plan.info["nchan"] or n_in > x.shape[1]:
            raise ValueError(f"beam {i}: input must be a uint8 CUDA tensor [nchan, >= n_in]")
        arr[i].plan = plan.handle.value
        arr[i].d_in = x.data_ptr()
        arr[i].in_pitch = x.stride(0)
        arr[i].n_in = int(n_in)
    dev = beams[0][1].device
    if work is None:
        work = torch.empty(int(work_bytes), dtype=torch.uint8, device=dev)
    cand = torch.empty(max(cap, 1) * 24 * n, dtype=torch.uint8, device=dev)
    count = torch.zeros(n, dtype=torch.int32, device=dev)
    info = N.BatchInfo()
    N.check(N.lib().aa_batch_run(arr, n, int(variant), _ptr(work), work.numel(), _ptr(cand), int(cap), _ptr(count),
                                 N.AA_BATCH_STATIC if static else 0, C.byref(info), _stream_handle(stream)))
    counts = count.cpu().numpy().astype(np.int64)
    out = []
    for i in range(n):   # only the filled part of each beam's slot comes to the host
        k = int(min(counts[i], cap))
        raw = cand[i * cap * 24:(i * cap + k) * 24].cpu().numpy()
        out.append(raw.view(N.CANDIDATE_DTYPE).copy())
    d = {k: getattr(info, k) for k, _ in N.BatchInfo._fields_}
    d["tune_ms"] = [float(v) for v in info.tune_ms][:N.lib().aa_variant_count()]
    return out, counts, d
