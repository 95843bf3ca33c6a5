"""Named synthetic workloads: sizes, band, DM plan, boxcars, threshold and pulses.

The names describe the content. Each entry is a plain dict. `make_input(w)` draws
the uint8 filterbank.

* tiny_128ch_32k: 128 channels x 32768 samples, f_top 1500 MHz, 0.78125 MHz
  channels, 64 us sampling, N(128, 16) noise. One pulse at DM 50 with FWHM
  4 samples and 3 sigma (48 counts) per channel, arriving at sample 20000.
  DM 0..99 in steps of 1, boxcars 1..32 (powers of two), S/N threshold 6.
* survey_4096ch_1M: 4096 channels x 2^20 samples, f_top 1450 MHz, 300 MHz band,
  64 us sampling, N(128, 16) noise. 20 pulses with DM U[10, 1500], FWHM
  log-U[1, 64] and amplitude U[0.1, 1] sigma per channel. 3000-trial doubling-step
  plan (0..1998), boxcars 1..256 (powers of two), threshold 6.
* streamed_128ch_8M: the tiny signal model at 2^23 samples. One DM-50 pulse per
  2^18-sample chunk, several of them placed on chunk and sub-chunk edges.
* survey_4096ch_1M_streamed: the survey signal fed in 2^18-sample chunks, where
  compute outweighs the PCIe transfer.
* batched_64beams and serving_32beams: see `batched_beams` and `serving_beams`.
"""

from __future__ import annotations

import numpy as np

from .dmplan import dm_plan, uniform_plan
from .filterbank import Pulse, arrival_offsets, make_filterbank, random_pulses

POW2_32 = [1, 2, 4, 8, 16, 32]
POW2_256 = [1, 2, 4, 8, 16, 32, 64, 128, 256]


def _tiny():
    return dict(name="tiny_128ch_32k", nchan=128, nsamp=32768, f_top=1500.0, foff=0.78125,
                tsamp=64e-6, dms=uniform_plan(100), widths=POW2_32, threshold=6.0,
                stat_block=32768, seed=1,
                pulses=[Pulse(dm=50.0, t0=20000.0, fwhm=4.0, amp=48.0)])


def _survey():
    nchan, nsamp, f_top, foff, tsamp = 4096, 1 << 20, 1450.0, 300.0 / 4096, 64e-6
    dms = dm_plan(3000)
    # keep every pulse (and its widest boxcar) inside the data at the bottom channel
    span = arrival_offsets(float(dms[-1]), nchan, f_top, foff, tsamp)[-1]
    t0_hi = nsamp - span - 256 - 200
    return dict(name="survey_4096ch_1M", nchan=nchan, nsamp=nsamp, f_top=f_top, foff=foff,
                tsamp=tsamp, dms=dms, widths=POW2_256, threshold=6.0, stat_block=32768, seed=2,
                pulses=random_pulses(20, seed=2, dm_range=(10.0, 1500.0), t0_range=(0.0, t0_hi)))


def _streamed():
    w = _tiny()
    nsamp, chunk = 1 << 23, 1 << 18
    # offsets inside each chunk: chunk edge, sub-chunk edges for 2/4/8 streams, interior
    offs = [0, 1, (1 << 15) - 2, 1 << 15, (1 << 16) - 1, (1 << 17) + 3, 100000, chunk - 3]
    pulses = [Pulse(50.0, 20000.0, 4.0, 48.0)]
    for k in range(1, nsamp // chunk - 1):
        pulses.append(Pulse(50.0, float(k * chunk + offs[k % len(offs)]), 4.0, 48.0))
    w.update(name="streamed_128ch_8M", nsamp=nsamp, chunk=chunk, streams=[1, 2, 4, 8],
             pulses=pulses, seed=3)
    return w


def _survey_streamed():
    w = _survey()
    w.update(name="survey_4096ch_1M_streamed", chunk=1 << 18, streams=[1, 2, 4, 8])
    return w


WORKLOADS = {"tiny_128ch_32k": _tiny, "survey_4096ch_1M": _survey, "streamed_128ch_8M": _streamed,
             "survey_4096ch_1M_streamed": _survey_streamed}


def workload(name: str) -> dict:
    return WORKLOADS[name]()


def make_input(w: dict, pitch: int | None = None, out=None, threads=None) -> np.ndarray:
    return make_filterbank(w["nchan"], w["nsamp"], w["f_top"], w["foff"], w["tsamp"],
                           w["pulses"], seed=w["seed"], pitch=pitch, out=out, threads=threads)


def batched_beams(nbeams: int = 64, seed: int = 4, nsamp_range=(1 << 16, 1 << 20),
                  ndm_range=(500, 3000), nchans=(1024, 2048, 4096)) -> list:
    """Uneven beams: nchan from `nchans`, nsamp and ndm uniform, 0-5 pulses each.
    Band and sampling are those of the survey workload (f_top 1450 MHz, 300 MHz, 64 us)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xBEA3]))
    beams = []
    for b in range(nbeams):
        nchan = int(rng.choice(nchans))
        nsamp = int(rng.integers(nsamp_range[0], nsamp_range[1] + 1))
        ndm = int(rng.integers(ndm_range[0], ndm_range[1] + 1))
        dms = dm_plan(ndm)
        foff = 300.0 / nchan
        span = arrival_offsets(float(dms[-1]), nchan, 1450.0, foff, 64e-6)[-1]
        npulse = int(rng.integers(0, 6))
        t0_hi = max(1.0, nsamp - span - 256 - 200)
        pulses = random_pulses(npulse, seed=seed * 1000 + b, dm_range=(min(10.0, dms[-1]), max(dms[-1] * 0.9, 1.0)),
                               t0_range=(0.0, t0_hi)) if npulse else []
        beams.append(dict(name=f"beam{b}", nchan=nchan, nsamp=nsamp, f_top=1450.0, foff=foff,
                          tsamp=64e-6, dms=dms, widths=POW2_256, threshold=6.0, stat_block=32768,
                          seed=seed * 1000 + b, pulses=pulses))
    return beams


def serving_beams(nbeams: int = 32, seed: int = 5, ndm_range=(500, 4096), rate_range=(0.5, 2.0)) -> list:
    """Beams of the serving workload: 4096 channels, 64 us, 2^17-sample chunks (8.39 s of
    sky each), ndm uniform in `ndm_range` (doubling-step plan), and a Poisson arrival rate
    of U[0.5, 2] times real time per beam."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5E4F]))
    out = []
    for b in range(nbeams):
        ndm = int(rng.integers(ndm_range[0], ndm_range[1] + 1))
        out.append(dict(name=f"beam{b}", nchan=4096, f_top=1450.0, foff=300.0 / 4096, tsamp=64e-6,
                        dms=dm_plan(ndm), widths=POW2_256, threshold=6.0, stat_block=32768,
                        rate=float(rng.uniform(*rate_range)), chunk=1 << 17))
    return out


def poisson_arrivals(beams: list, duration_s: float, seed: int = 6, rate_scale: float = 1.0) -> list:
    """Sorted (time_s, beam) arrivals. Beam b emits a chunk every chunk*tsamp/rate seconds
    on average (exponential gaps)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xA771]))
    ev = []
    for i, b in enumerate(beams):
        lam = b["rate"] * rate_scale / (b["chunk"] * b["tsamp"])
        t = float(rng.exponential(1.0 / lam))
        while t < duration_s:
            ev.append((t, i))
            t += float(rng.exponential(1.0 / lam))
    ev.sort()
    return ev
