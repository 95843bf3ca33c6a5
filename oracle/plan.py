"""Shift table and sizes (the "mapping tasks to resources" step of the paper's
workflow, section 1, where all sizes and allocations are fixed before the search).

Readings where the paper is silent:
* Channel c has centre frequency f_c = f_top - c * foff. Channel 0 is the highest,
  so its shift is 0 for every DM.
* The dispersion constant is K = 4.148808e3 MHz^2 s per (pc cm^-3).
* s[d][c] = floor(((K * DM_d) * (1/(f_c*f_c) - 1/(f_top*f_top))) / t_samp + 0.5).
  Every operation is one IEEE float64 operation, in exactly this order and with no
  fused multiply-add.
* maxshift M = max s. The dedispersed length is N_dd = nsamp - M ("valid only",
  with no zero padding). The number of boxcar starts is T = N_dd - wmax + 1.
"""

import numpy as np

K_DM = 4.148808e3


def channel_freqs(nchan: int, f_top: float, foff: float) -> np.ndarray:
    """f_c = f_top - c * foff (float64, one multiply then one subtract)."""
    c = np.arange(nchan, dtype=np.float64)
    return np.float64(f_top) - c * np.float64(foff)


def shift_table(dms, nchan: int, f_top: float, foff: float, tsamp: float) -> np.ndarray:
    """Integer sample shift of channel c at DM trial d, as int64 [ndm, nchan]."""
    dms = np.asarray(dms, dtype=np.float64)
    f = channel_freqs(nchan, f_top, foff)
    ftop = np.float64(f_top)
    inv = 1.0 / (f * f) - 1.0 / (ftop * ftop)          # per channel
    kdm = np.float64(K_DM) * dms                       # per trial
    x = (kdm[:, None] * inv[None, :]) / np.float64(tsamp) + 0.5
    return np.floor(x).astype(np.int64)


def sizes(shifts: np.ndarray, nsamp: int, widths, stat_block: int) -> dict:
    """Plan-wide sizes: maxshift, N_dd, T (starts) and the number of stat blocks."""
    m = int(shifts.max())
    wmax = int(max(widths))
    n_dd = nsamp - m
    n_start = n_dd - wmax + 1
    nblocks = -(-n_start // stat_block) if n_start > 0 else 0
    return dict(maxshift=m, n_dd=n_dd, n_start=n_start, wmax=wmax, nblocks=nblocks)
