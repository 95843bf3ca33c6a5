"""Seeded uint8 filterbank generator: Gaussian noise plus dispersed Gaussian pulses.

Signal model:
* Channel c has centre frequency f_top - c * foff (MHz). Channel 0 is the highest.
* Noise is N(mean, sigma) per sample, drawn as float32 from channel c's own child
  stream of `SeedSequence(seed)`. Rows are therefore reproducible, and they can be
  generated in parallel in any order.
* A pulse has a DM, an arrival sample t0 at the top channel, a FWHM in samples and
  a peak amplitude in counts per channel. In channel c it is a Gaussian centred on
  t0 + delay_c. delay_c is the cold-plasma dispersion delay of channel c relative
  to the top channel: 4.148808 ms * DM * ((f_c/GHz)^-2 - (f_top/GHz)^-2), converted
  to samples and left unrounded.
* The sum is rounded half-to-even, clipped to [0, 255] and stored as uint8.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

# Dispersion constant of the signal model, in ms GHz^2 per (pc cm^-3).
_DISPERSION_MS_GHZ2 = 4.148808
_FWHM_PER_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))


@dataclass(frozen=True)
class Pulse:
    dm: float      # pc cm^-3
    t0: float      # arrival sample at the top channel (may be fractional)
    fwhm: float    # samples
    amp: float     # peak counts added per channel


def arrival_offsets(dm: float, nchan: int, f_top: float, foff: float, tsamp: float) -> np.ndarray:
    """Continuous arrival delay (samples) of a pulse of dispersion `dm` in every channel."""
    f_ghz = (f_top - np.arange(nchan, dtype=np.float64) * foff) / 1000.0
    ftop_ghz = f_top / 1000.0
    delay_ms = _DISPERSION_MS_GHZ2 * dm * (f_ghz ** -2 - ftop_ghz ** -2)
    return delay_ms * 1e-3 / tsamp


def _row(c, child, nsamp, f_top, foff, tsamp, pulses, offsets, mean, sigma, out_row):
    rng = np.random.default_rng(child)
    x = rng.standard_normal(nsamp, dtype=np.float32)
    x *= np.float32(sigma)
    x += np.float32(mean)
    for p, off in zip(pulses, offsets):
        centre = p.t0 + off[c]
        sd = p.fwhm / _FWHM_PER_SIGMA
        lo = max(0, int(math.floor(centre - 6.0 * sd)) - 1)
        hi = min(nsamp, int(math.ceil(centre + 6.0 * sd)) + 2)
        if lo >= hi:
            continue
        t = np.arange(lo, hi, dtype=np.float64)
        x[lo:hi] += (p.amp * np.exp(-0.5 * ((t - centre) / sd) ** 2)).astype(np.float32)
    np.rint(x, out=x)
    np.clip(x, 0.0, 255.0, out=x)
    out_row[:nsamp] = x.astype(np.uint8)


def make_filterbank(nchan: int, nsamp: int, f_top: float, foff: float, tsamp: float,
                    pulses=(), seed: int = 0, mean: float = 128.0, sigma: float = 16.0,
                    pitch: int | None = None, out: np.ndarray | None = None,
                    threads: int | None = None) -> np.ndarray:
    """Return (or fill `out` with) a uint8 array [nchan, pitch].

    Columns past `nsamp` are left as they are in `out`, or zero in a new array.
    """
    pitch = nsamp if pitch is None else pitch
    if pitch < nsamp:
        raise ValueError("pitch must be >= nsamp")
    if out is None:
        out = np.zeros((nchan, pitch), dtype=np.uint8)
    elif out.shape[0] < nchan or out.shape[1] < nsamp or out.dtype != np.uint8:
        raise ValueError("out has the wrong shape or dtype")
    pulses = list(pulses)
    offsets = [arrival_offsets(p.dm, nchan, f_top, foff, tsamp) for p in pulses]
    children = np.random.SeedSequence(seed).spawn(nchan)
    threads = threads or min(16, os.cpu_count() or 1)

    def work(c):
        _row(c, children[c], nsamp, f_top, foff, tsamp, pulses, offsets, mean, sigma, out[c])

    if nchan * nsamp < (1 << 22) or threads == 1:
        for c in range(nchan):
            work(c)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(nchan)))
    return out


def random_pulses(n: int, seed: int, dm_range, t0_range, fwhm_range=(1.0, 64.0),
                  amp_range=(0.1 * 16.0, 16.0)) -> list:
    """`n` pulses. DM and t0 are uniform, FWHM is log-uniform and amplitude is uniform."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x9E3779B9]))
    dms = rng.uniform(dm_range[0], dm_range[1], n)
    t0s = rng.uniform(t0_range[0], t0_range[1], n)
    fw = np.exp(rng.uniform(math.log(fwhm_range[0]), math.log(fwhm_range[1]), n))
    amps = rng.uniform(amp_range[0], amp_range[1], n)
    return [Pulse(float(d), float(t), float(w), float(a)) for d, t, w, a in zip(dms, t0s, fw, amps)]
