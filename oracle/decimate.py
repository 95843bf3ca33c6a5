"""Per-range time decimation (a form that goes beyond the paper: its dedispersion phase,
section 2.1, is brute force at the input resolution; the doubling DM step of the survey
plan suggests halving the time resolution with each doubling of the step, which keeps the
bottom channel's shift step per trial near one sample while cutting the adds).

TEST INFRASTRUCTURE, like the rest of `oracle/`: plain and slow, no shared code with the
GPU library.

Definitions (readings, since the paper gives none):
* Decimation by 2 of a uint8 row is the rounding average of adjacent pairs,
      y[j] = (x[2j] + x[2j+1] + 1) >> 1,   0 <= j < floor(n / 2),
  exact in integers; a trailing odd sample is dropped. Decimation by f = 2^k applies
  this k times (not the rounded mean of f samples: each halving rounds).
* A range plan splits the trials into consecutive ranges r = 0, 1, ... with first
  trial a_r (a_0 = 0) and factor f_r (powers of two, non-decreasing). Range r is an
  ordinary plan over the input decimated by f_r, with sampling time f_r * t_samp
  (one exact float64 product), the range's trials, stat blocks of B / f_r of its
  samples, the same widths (in its samples) and threshold. Its maxshift, N_dd and T
  are its own.
* The range's candidates come from its own plane: the 3x3 peak test sees only the
  range's trials (the first and last trial of a range have no neighbour across the
  range edge). A candidate is reported as (global trial index, f_r * j, f_r * w, S/N):
  its start and width in input samples.
* The list over all ranges is sorted by (trial, start); ranges are in trial order, so
  this is the concatenation of the ranges' lists.
"""

from __future__ import annotations

import numpy as np

from .dedisp import dedisperse
from .plan import shift_table, sizes
from .sps import single_pulse


def decimate2(x: np.ndarray, n: int | None = None) -> np.ndarray:
    """Rounding average of adjacent sample pairs along each row (uint8 -> uint8)."""
    n = x.shape[1] if n is None else n
    m = n // 2
    a = x[:, 0:2 * m:2].astype(np.int64)
    b = x[:, 1:2 * m:2].astype(np.int64)
    return ((a + b + 1) >> 1).astype(np.uint8)


def decimate(x: np.ndarray, f: int, n: int | None = None) -> np.ndarray:
    """Decimation by f = 2^k: k successive halvings."""
    if f < 1 or f & (f - 1):
        raise ValueError("the decimation factor must be a power of two")
    y = x[:, : (x.shape[1] if n is None else n)]
    while f > 1:
        y = decimate2(y)
        f //= 2
    return np.ascontiguousarray(y)


def check_ranges(ndm: int, first, factor, stat_block: int):
    first = [int(a) for a in first]
    factor = [int(f) for f in factor]
    if not first or first[0] != 0 or len(first) != len(factor):
        raise ValueError("ranges must start at trial 0, one factor per range")
    if any(b <= a for a, b in zip(first, first[1:] + [ndm])):
        raise ValueError("range first trials must ascend below ndm")
    if any(f < 1 or f & (f - 1) for f in factor) or any(g < f for f, g in zip(factor, factor[1:])):
        raise ValueError("factors must be non-decreasing powers of two")
    if any(stat_block % f for f in factor):
        raise ValueError("every factor must divide the stat block")
    return first, factor


def range_plans(dms, nchan, nsamp, f_top, foff, tsamp, widths, stat_block, first, factor):
    """Per range: trials [lo, hi), factor f, shift table, sizes, decimated length n."""
    dms = np.asarray(dms, dtype=np.float64)
    first, factor = check_ranges(len(dms), first, factor, stat_block)
    out = []
    for r, (lo, f) in enumerate(zip(first, factor)):
        hi = first[r + 1] if r + 1 < len(first) else len(dms)
        n = nsamp
        g = f
        while g > 1:
            n //= 2
            g //= 2
        s = shift_table(dms[lo:hi], nchan, f_top, foff, np.float64(f) * np.float64(tsamp))
        out.append(dict(lo=lo, hi=hi, f=f, shifts=s, n=n, block=stat_block // f,
                        sizes=sizes(s, n, widths, stat_block // f)))
    return out


def run_ranges(x, nsamp, f_top, foff, tsamp, dms, widths, threshold, stat_block, first, factor):
    """All ranges: decimate, dedisperse, search; candidates in input samples."""
    plans = range_plans(dms, x.shape[0], nsamp, f_top, foff, tsamp, widths, stat_block, first, factor)
    cands = []
    for rp in plans:
        xd = decimate(x, rp["f"], nsamp)
        sz = rp["sizes"]
        if sz["n_start"] < 1:
            raise ValueError(f"range at trial {rp['lo']} is too short after decimation")
        D = dedisperse(xd, rp["shifts"], rp["n"], sz["maxshift"])
        T = sz["n_start"]
        c, _ = single_pulse(D, 0, 0, T, T, widths, threshold, rp["block"])
        f = rp["f"]
        cands.extend((rp["lo"] + d, f * t, f * w, snr) for d, t, w, snr in c)
    cands.sort(key=lambda c: (c[0], c[1]))
    return dict(plans=plans, candidates=cands)
