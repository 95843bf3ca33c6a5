"""ctypes view of the C ABI in include/aa.h. Argument marshalling only.

Importing this module loads the in-tree libaa_mi355x.so. If the library has not
been built, it raises ImportError. There is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libaa_mi355x.so")

AA_OK, AA_EAGAIN, AA_EINVAL, AA_ESHORT, AA_ENOMEM, AA_EHIP, AA_EOVERFLOW, AA_EBUSY = 0, 1, -1, -2, -3, -4, -5, -6
AA_PLAN_HOST_ONLY = 1
STATUS_NAMES = {0: "AA_OK", 1: "AA_EAGAIN", -1: "AA_EINVAL", -2: "AA_ESHORT", -3: "AA_ENOMEM",
                -4: "AA_EHIP", -5: "AA_EOVERFLOW", -6: "AA_EBUSY"}

CANDIDATE_DTYPE = np.dtype([("dm_idx", "<i4"), ("width", "<i4"), ("t", "<i8"), ("snr", "<f4"), ("beam", "<i4")])
assert CANDIDATE_DTYPE.itemsize == 24


class PlanDesc(C.Structure):
    _fields_ = [("nchan", C.c_int32), ("nsamp", C.c_int64), ("f_top_mhz", C.c_double),
                ("foff_mhz", C.c_double), ("tsamp_s", C.c_double), ("dm", C.POINTER(C.c_double)),
                ("ndm", C.c_int32), ("widths", C.POINTER(C.c_int32)), ("nwidths", C.c_int32),
                ("snr_threshold", C.c_float), ("stat_block", C.c_int32), ("flags", C.c_uint32),
                ("clip_sigma", C.c_float), ("clip_iters", C.c_int32), ("boxcar_full_width", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("nchan", C.c_int32), ("ndm", C.c_int32), ("nwidths", C.c_int32), ("wmax", C.c_int32),
                ("nsamp", C.c_int64), ("maxshift", C.c_int64), ("n_dd", C.c_int64), ("n_start", C.c_int64),
                ("stat_block", C.c_int64), ("nblocks", C.c_int64), ("in_pitch", C.c_int64),
                ("out_pitch", C.c_int64), ("work_bytes", C.c_size_t), ("device", C.c_int32)]


class VariantInfo(C.Structure):
    _fields_ = [("id", C.c_int32), ("waves", C.c_int32), ("dm_per_wave", C.c_int32),
                ("trials_per_block", C.c_int32), ("lds_bytes", C.c_int32), ("layout", C.c_int32),
                ("time_tile", C.c_int32), ("depth", C.c_int32), ("max_tiles", C.c_int32)]


class PipelineOpts(C.Structure):
    _fields_ = [("nstreams", C.c_int32), ("max_beams", C.c_int32), ("max_chunk", C.c_int64),
                ("cand_cap", C.c_int32), ("result_slots", C.c_int32), ("hbm_budget", C.c_int64),
                ("flags", C.c_uint32), ("min_piece_work", C.c_int64)]


class Result(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("beam", C.c_int32), ("status", C.c_int32), ("t_begin", C.c_int64),
                ("t_end", C.c_int64), ("n_true", C.c_int64), ("n", C.c_int64), ("cand", C.c_void_p),
                ("latency_s", C.c_double), ("queue_s", C.c_double)]


class PipelineStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("in_flight", C.c_int64),
                ("queued", C.c_int64), ("arena_bytes", C.c_int64), ("arena_used", C.c_int64),
                ("arena_peak", C.c_int64), ("copy_ms", C.c_double), ("kernel_ms", C.c_double),
                ("overlap_ms", C.c_double), ("span_ms", C.c_double), ("copy_sum_ms", C.c_double),
                ("kernel_sum_ms", C.c_double)]


AA_PIPE_SERIAL, AA_PIPE_TIMING, AA_PIPE_SDMA_COPY, AA_PIPE_STAGED, AA_SUBMIT_LAST = 1, 2, 4, 8, 1
AA_BATCH_STATIC = 1


class BatchBeam(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("d_in", C.c_void_p), ("in_pitch", C.c_int64), ("n_in", C.c_int64)]


class BatchInfo(C.Structure):
    _fields_ = [("groups", C.c_int32), ("variant", C.c_int32), ("items", C.c_int64), ("ms_dedisp", C.c_float),
                ("ms_search", C.c_float), ("tuned_beam", C.c_int32), ("tune_ms", C.c_float * 32)]


CLUSTER_DTYPE = np.dtype([("peak", CANDIDATE_DTYPE), ("members", "<i4"), ("dm_lo", "<i4"), ("dm_hi", "<i4"),
                          ("pad", "<i4"), ("t_lo", "<i8"), ("t_hi", "<i8")])
assert CLUSTER_DTYPE.itemsize == 56


class AAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2101_00941_amd.build` "
                          "(or __graft_entry__.build())")
    # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7. Loading torch
    # first makes the library's libamdhip64.so.7 dependency bind to that same copy
    # (same soname), instead of mapping a second runtime from /opt/rocm.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    sig = {
        "aa_last_error": (C.c_char_p, []),
        "aa_version": (C.c_char_p, []),
        "aa_plan": (C.c_int, [C.POINTER(PlanDesc), C.POINTER(vp)]),
        "aa_plan_info": (C.c_int, [vp, C.POINTER(PlanInfo)]),
        "aa_plan_shifts": (C.c_int, [vp, vp]),
        "aa_plan_destroy": (None, [vp]),
        "aa_dedisperse": (C.c_int, [vp, vp, i64, i64, vp, i64, vp]),
        "aa_single_pulse_work_bytes": (C.c_int, [vp, i64, C.POINTER(sz)]),
        "aa_variant_count": (C.c_int, []),
        "aa_variant_info": (C.c_int, [i32, C.POINTER(VariantInfo)]),
        "aa_plan_set_variant": (C.c_int, [vp, i32]),
        "aa_plan_get_variant": (C.c_int, [vp, C.POINTER(i32)]),
        "aa_autotune": (C.c_int, [vp, vp, i64, i64, vp, i64, i32, vp, C.POINTER(C.c_float)]),
        "aa_pipeline_create": (C.c_int, [C.POINTER(PipelineOpts), C.POINTER(vp)]),
        "aa_pipeline_add_beam": (C.c_int, [vp, vp, C.POINTER(i32)]),
        "aa_pipeline_add_beam_at": (C.c_int, [vp, vp, i64, C.POINTER(i32)]),
        "aa_stream_submit": (C.c_int, [vp, i32, vp, i64, i64, C.c_uint64, C.c_uint32]),
        "aa_poll": (C.c_int, [vp, C.POINTER(Result), i32]),
        "aa_release": (C.c_int, [vp, C.c_uint64]),
        "aa_pipeline_stats": (C.c_int, [vp, C.POINTER(PipelineStats)]),
        "aa_pipeline_destroy": (C.c_int, [vp]),
        "aa_batch_run": (C.c_int, [C.POINTER(BatchBeam), i32, i32, vp, sz, vp, i32, vp, C.c_uint32,
                                   C.POINTER(BatchInfo), vp]),
        "aa_single_pulse": (C.c_int, [vp, vp, i64, i64, i64, i64, i64, i64, vp, sz, vp, i32, vp, vp, i64, vp]),
        "aa_single_pulse_noalloc": (C.c_int, [vp, vp, i64, i64, i64, i64, i64, i64, vp, i32, vp, vp, i64, vp]),
        "aa_decimate2": (C.c_int, [vp, i64, i64, i32, vp, i64, vp]),
        "aa_cluster": (C.c_int, [vp, i64, i32, i64, vp, i64, C.POINTER(i64)]),
        "aa_range_plan": (C.c_int, [C.POINTER(PlanDesc), C.POINTER(i32), C.POINTER(i32), i32, C.POINTER(vp)]),
        "aa_range_plan_get": (C.c_int, [vp, i32, C.POINTER(vp), C.POINTER(i32), C.POINTER(i32)]),
        "aa_range_work_bytes": (C.c_int, [vp, i64, i32, C.POINTER(sz)]),
        "aa_range_run": (C.c_int, [vp, vp, i64, i64, vp, sz, vp, i32, vp, vp]),
        "aa_range_autotune": (C.c_int, [vp, vp, i64, i64, vp, sz, i32, vp, C.POINTER(C.c_float)]),
        "aa_range_plan_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(rc: int) -> int:
    if rc < 0:
        raise AAError(rc, lib().aa_last_error().decode())
    return rc
