"""Brute-force incoherent dedispersion (the paper's dedispersion phase, section 2.1).

Definition: D[d][t] = sum over c < nchan of X[c][t + s[d][c]], for 0 <= t < n_out,
where n_out = n_in - maxshift. X is uint8. D is accumulated exactly in int32, since
at most 65535 * 255 < 2^31, and returned as int64.
A DM-0 trial has all shifts 0, so it is the plain channel sum.
"""

import numpy as np


def dedisperse(x: np.ndarray, shifts: np.ndarray, n_in: int | None = None, maxshift: int | None = None) -> np.ndarray:
    """All DM rows. `x` is uint8 [nchan, >= n_in], `shifts` int [ndm, nchan]."""
    return dedisperse_rows(x, shifts, range(shifts.shape[0]), n_in, maxshift)


def dedisperse_rows(x: np.ndarray, shifts: np.ndarray, rows, n_in: int | None = None,
                    maxshift: int | None = None) -> np.ndarray:
    """Only the DM rows listed in `rows`, in that order. Returns int64 [len(rows), n_out]."""
    nchan = shifts.shape[1]
    if x.shape[0] < nchan:
        raise ValueError("input has fewer channels than the shift table")
    n_in = x.shape[1] if n_in is None else n_in
    m = int(shifts.max()) if maxshift is None else maxshift
    n_out = n_in - m
    if n_out < 1:
        raise ValueError("input shorter than maxshift + 1")
    rows = list(rows)
    if nchan > 65535:
        raise ValueError("more than 65535 channels could overflow int32 sums")
    out = np.zeros((len(rows), n_out), dtype=np.int64)
    acc = np.zeros(n_out, dtype=np.int32)
    for i, d in enumerate(rows):
        acc[:] = 0
        for c in range(nchan):
            s = int(shifts[d, c])
            np.add(acc, x[c, s:s + n_out], out=acc)
        out[i] = acc
    return out
