"""Whole-signal and chunked oracle runs.

Section 1 of the paper splits the input into time chunks that fit in GPU memory.
Section 2 splits each chunk again, once per stream. The reading used for chunk
edges is this. A chunk covers the starts [a, b), with a a multiple of the stat
block. It reads the input samples [a - 1, b + wmax + M), clipped to the signal.
Consecutive windows therefore overlap by M + wmax + 1 samples. That overlap gives
the chunk the left and right neighbour columns that the 3x3 peak test needs, and
the full width of the last boxcars. With this reading the chunked result equals
the whole-signal result exactly.
"""

import numpy as np

from .dedisp import dedisperse
from .plan import shift_table, sizes
from .sps import single_pulse


def run(x, nsamp, f_top, foff, tsamp, dms, widths, threshold, stat_block=32768, want_best=False, clip_sigma=0.0,
        clip_iters=0, boxcar_full_width=0):
    """Dedisperse all trials, then run the single-pulse search over every start."""
    s = shift_table(dms, x.shape[0], f_top, foff, tsamp)
    sz = sizes(s, nsamp, widths, stat_block)
    D = dedisperse(x, s, nsamp, sz["maxshift"])
    T = sz["n_start"]
    cands, best = single_pulse(D, 0, 0, T, T, widths, threshold, stat_block, want_best=want_best,
                               clip_sigma=clip_sigma, clip_iters=clip_iters, boxcar_full_width=boxcar_full_width)
    return dict(shifts=s, sizes=sz, D=D, candidates=cands, best=best)


def run_chunked(x, nsamp, f_top, foff, tsamp, dms, widths, threshold, chunk, stat_block=32768, clip_sigma=0.0,
                clip_iters=0, boxcar_full_width=0):
    """Same result as `run`, computed one chunk of `chunk` starts at a time."""
    if chunk % stat_block:
        raise ValueError("chunk must be a multiple of the stat block")
    s = shift_table(dms, x.shape[0], f_top, foff, tsamp)
    sz = sizes(s, nsamp, widths, stat_block)
    m, wmax, T = sz["maxshift"], sz["wmax"], sz["n_start"]
    out = []
    for a in range(0, T, chunk):
        b = min(a + chunk, T)
        lo = max(a - 1, 0)
        hi = min(b + wmax + m, nsamp)
        D = dedisperse(np.ascontiguousarray(x[:, lo:hi]), s, hi - lo, m)
        c, _ = single_pulse(D, lo, a, b, T, widths, threshold, stat_block, clip_sigma=clip_sigma,
                            clip_iters=clip_iters, boxcar_full_width=boxcar_full_width)
        out.extend(c)
    out.sort(key=lambda c: (c[0], c[1]))
    return out
