"""Single-pulse search on a dedispersed plane (the paper's SPDT phase, section 2.2).

The paper names the phase but defers its algorithm to its reference on single-pulse
detection. The definition used here is the boxcar S/N search it describes, with
these readings:

* Boxcar: the start-aligned window sum_w(d, t) = sum over i < w of D[d][t + i],
  for the starts 0 <= t < T. The reported t is the start sample.
* Statistics: per DM row and per stat block of B consecutive starts (blocks are
  aligned to absolute start 0, and the last one may be partial). With n, S1 and S2
  the exact count, sum and sum of squares over the block's starts:
      mu      = S1 / n                           (one rounding)
      var     = fl(n*S2 - S1^2) / (n*n)          (exact integer, then two roundings)
      sigma   = sqrt(var)                        (population std)
* Optional outlier clipping (clip_iters > 0 and clip_sigma > 0; robust statistics in
  the spirit of the single-pulse search the paper cites): starting from all of the
  block's values, each iteration computes mu and sigma as above from the values kept
  so far, then keeps the block's values D with |float(D) - mu| <= c * sigma, where
  c = float64(float32(clip_sigma)) and the product is one rounding; n, S1 and S2 are
  then recomputed exactly over the kept values. If an iteration would keep no value,
  the previous moments stay and clipping stops. The normalisation below uses the final
  moments; the window sums and S/N are over all values, as without clipping.
* Normalisation per block and width: wmu_w = w * mu and r_w = 1 / (sigma * sqrt(w)),
  where sqrt(w) is rounded first. If sigma == 0 then r_w = 0, so that S/N is 0.
* S/N(d, t, w) = (float(sum_w) - wmu_w) * r_w. This is (sum - w mu) / (sigma sqrt w)
  with the rounding points fixed.
* best(d, t) = max over w of S/N. wbest is the smallest width that attains it.
* Optional decimated boxcar hierarchy (boxcar_full_width w0 > 0; the single-pulse search
  the paper cites reaches wide boxcars on decimated data, where a width-w' boxcar over
  sums of 2^l adjacent samples is the width-2^l w' boxcar of the plane at a start that is a
  multiple of 2^l): width w is evaluated at the starts t that are multiples of its stride
  s(w), the smallest power of two with w0 * s(w) >= w (s = 1 for w <= w0). The window
  sums are unchanged, only the starts at which wide widths are tried are thinned. best and
  wbest are over the widths evaluated at t; the first width must be <= w0.
* Peak: (d, t) is a candidate iff best >= threshold and best is a 3x3 local maximum
  in (DM index, start). It must be strictly greater than the neighbours that come
  earlier in row-major (d, t) order, and >= the later ones. Neighbours outside
  [0, ndm) x [0, T) do not count. Every value in the 3x3 window is normalised with
  the statistics of the centre's block, each in its own DM row.
* Output: (dm_idx, t, width, float32(best)), sorted by (dm_idx, t).
"""

from __future__ import annotations

import math

import numpy as np


def block_moments(seg: np.ndarray):
    """Exact (n, S1, S2) per row over the columns of `seg` (int64 [rows, n])."""
    n = seg.shape[1]
    s1 = [int(v) for v in seg.sum(axis=1, dtype=np.int64)]
    s2 = [int(v) for v in (seg.astype(np.int64) ** 2).sum(axis=1, dtype=np.int64)]
    if seg.size and int(seg.max()) ** 2 * n >= 2 ** 63:
        raise OverflowError("block sum of squares exceeds int64")
    return n, s1, s2


def clipped_moments(seg: np.ndarray, clip_sigma: float, clip_iters: int):
    """Per row: exact (n, S1, S2) after the clipping iterations of the module header."""
    c = float(np.float32(clip_sigma))
    ns, s1s, s2s = [], [], []
    for row in seg.astype(np.int64):
        n, a, b = row.size, int(row.sum()), int((row * row).sum())
        for _ in range(clip_iters):
            mu = a / n
            sigma = math.sqrt(float(n * b - a * a) / float(n * n))
            keep = row[np.abs(row.astype(np.float64) - mu) <= c * sigma]
            if keep.size == 0:
                break
            n, a, b = keep.size, int(keep.sum()), int((keep * keep).sum())
        ns.append(n)
        s1s.append(a)
        s2s.append(b)
    return ns, s1s, s2s


def block_norms(n, s1: list, s2: list, widths):
    """Per row: (wmu [nw], r [nw]) as float64, following the module's rounding rules.
    n is the count shared by every row, or one count per row."""
    nw = len(widths)
    wmu = np.zeros((len(s1), nw))
    r = np.zeros((len(s1), nw))
    sqrtw = [math.sqrt(float(w)) for w in widths]
    nrow = [n] * len(s1) if isinstance(n, (int, np.integer)) else list(n)
    for i, (a, b, n) in enumerate(zip(s1, s2, nrow)):
        mu = a / n                                   # exact rational, one rounding
        var = float(n * b - a * a) / float(n * n)
        sigma = math.sqrt(var)
        for k, w in enumerate(widths):
            wmu[i, k] = float(w) * mu
            r[i, k] = 0.0 if sigma == 0.0 else 1.0 / (sigma * sqrtw[k])
    return wmu, r


def boxcar_strides(widths, full_width: int):
    """Stride of each width under the decimated boxcar hierarchy (all 1 if full_width is 0)."""
    out = []
    for w in widths:
        s = 1
        if full_width > 0:
            while full_width * s < w:
                s *= 2
        out.append(s)
    return out


def best_plane(prefix: np.ndarray, col0: int, lo: int, hi: int, widths, wmu, r, strides=None):
    """best and wbest index for the starts [lo, hi). Row i uses wmu[i] and r[i].

    `prefix[:, k]` = sum of the first k plane columns, and plane column 0 is absolute
    start `col0`. strides: width k is tried only at starts that are multiples of
    strides[k] (none: every start).
    """
    a = lo - col0
    best = None
    widx = None
    starts = np.arange(lo, hi)
    for k, w in enumerate(widths):
        ssum = prefix[:, a + w:hi - col0 + w] - prefix[:, a:hi - col0]
        snr = (ssum.astype(np.float64) - wmu[:, k:k + 1]) * r[:, k:k + 1]
        if strides is not None and strides[k] > 1:
            snr = np.where((starts % strides[k] == 0)[None, :], snr, -np.inf)
        if best is None:
            best = snr
            widx = np.zeros(snr.shape, dtype=np.int64)
        else:
            upd = snr > best
            best = np.where(upd, snr, best)
            widx = np.where(upd, k, widx)
    return best, widx


def candidates(center, v_prev, v_same, v_next, threshold):
    """Boolean peak mask for `center` (row d, starts [b0, b1)).

    `v_prev`, `v_same` and `v_next` hold rows d-1, d and d+1 over starts
    [b0 - 1, b1 + 1), with -inf where the neighbour is out of range.
    """
    n = center.shape[0]
    ok = center >= threshold
    # earlier in row-major order: every start of row d-1, and (d, t-1): strictly greater
    for dt in (0, 1, 2):
        ok &= center > v_prev[dt:dt + n]
    ok &= center > v_same[0:n]
    # later: (d, t+1) and every start of row d+1: greater or equal
    ok &= center >= v_same[2:2 + n]
    for dt in (0, 1, 2):
        ok &= center >= v_next[dt:dt + n]
    return ok


def single_pulse(D: np.ndarray, dd_t0: int, t_begin: int, t_end: int, t_total: int, widths,
                 threshold: float, stat_block: int, row0: int = 0, ndm: int | None = None,
                 report_rows=None, want_best: bool = False, clip_sigma: float = 0.0, clip_iters: int = 0,
                 boxcar_full_width: int = 0):
    """Candidates for the starts [t_begin, t_end) of a dedispersed plane.

    D: int64 [nrows, ncols]. Row i is DM trial row0 + i, and column j is absolute
       sample dd_t0 + j.
    t_begin must be a multiple of `stat_block`. t_total is the total number of starts
    T of the whole signal, or -1 if the columns after t_end are real data.
    report_rows: DM indices to report. By default these are all rows whose two
    neighbour rows are either present in D or outside [0, ndm).
    Returns (list of (d, t, width, snr_f32) sorted by (d, t), best plane or None).
    """
    widths = [int(w) for w in widths]
    strides = boxcar_strides(widths, boxcar_full_width)
    if strides[0] != 1:
        raise ValueError("the first width must not exceed boxcar_full_width")
    nrows = D.shape[0]
    ndm = row0 + nrows if ndm is None else ndm
    wmax = max(widths)
    if t_begin % stat_block:
        raise ValueError("t_begin must be a multiple of the stat block")
    if t_begin - 1 >= 0 and dd_t0 > t_begin - 1:
        raise ValueError("plane lacks the left halo column")
    right = t_end if (t_total >= 0 and t_end >= t_total) else t_end + 1
    if dd_t0 + D.shape[1] < right + wmax - 1:
        raise ValueError("plane too short for the boxcars at the right edge")
    if report_rows is None:
        report_rows = [row0 + i for i in range(nrows)
                       if (i > 0 or row0 == 0) and (i < nrows - 1 or row0 + nrows == ndm)]
    for d in report_rows:
        i = d - row0
        if not (0 <= i < nrows) or (i == 0 and d > 0) or (i == nrows - 1 and d + 1 < ndm):
            raise ValueError(f"row {d} or one of its neighbour rows is not in the plane")
    prefix = np.zeros((nrows, D.shape[1] + 1), dtype=np.int64)
    np.cumsum(D, axis=1, out=prefix[:, 1:])
    neg = -np.inf
    out = []
    best_out = np.zeros((nrows, t_end - t_begin), dtype=np.float32) if want_best else None
    for b0 in range(t_begin, t_end, stat_block):
        b1 = min(b0 + stat_block, t_end)
        if clip_iters > 0 and clip_sigma > 0:
            n, s1, s2 = clipped_moments(D[:, b0 - dd_t0:b1 - dd_t0], clip_sigma, clip_iters)
        else:
            n, s1, s2 = block_moments(D[:, b0 - dd_t0:b1 - dd_t0])
        wmu, r = block_norms(n, s1, s2, widths)
        lo = max(b0 - 1, 0)
        hi = b1 + 1 if (t_total < 0 or b1 + 1 <= t_total) else t_total
        v, widx = best_plane(prefix, dd_t0, lo, hi, widths, wmu, r, strides)
        # pad to starts [b0 - 1, b1 + 1) with -inf outside the range of starts
        pad = np.full((nrows, (b1 + 1) - (b0 - 1)), neg)
        pad[:, lo - (b0 - 1):hi - (b0 - 1)] = v
        if want_best:
            best_out[:, b0 - t_begin:b1 - t_begin] = v[:, b0 - lo:b1 - lo].astype(np.float32)
        empty = np.full(pad.shape[1], neg)
        for d in report_rows:
            i = d - row0
            prev_row = pad[i - 1] if d - 1 >= 0 else empty
            next_row = pad[i + 1] if d + 1 < ndm else empty
            same = pad[i]
            center = same[1:1 + (b1 - b0)]
            ok = candidates(center, prev_row, same, next_row, threshold)
            for j in np.flatnonzero(ok):
                t = b0 + int(j)
                out.append((d, t, widths[int(widx[i, t - lo])], float(np.float32(center[j]))))
    out.sort(key=lambda c: (c[0], c[1]))
    return out, best_out
