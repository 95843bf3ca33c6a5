"""Device-side variant of the seeded filterbank generator, for workloads too large
to draw on the host (tens of GB). It uses the same signal model as `filterbank.py`:
N(mean, sigma) noise plus dispersed Gaussian pulses, rounded half-to-even and
clipped to [0, 255]. The noise comes from torch's seeded device generator, so it
is reproducible on one device type but not bit-identical to the numpy generator.
To check a beam against the CPU oracle, copy that beam's generated input to the
host.
"""

from __future__ import annotations

import math

import numpy as np

from .filterbank import _FWHM_PER_SIGMA, arrival_offsets


def make_filterbank_torch(nchan, nsamp, f_top, foff, tsamp, pulses=(), seed=0, mean=128.0, sigma=16.0,
                          pitch=None, device="cuda", rows_per_step=256):
    import torch
    pitch = pitch or (nsamp + 255) // 256 * 256
    out = torch.zeros((nchan, pitch), dtype=torch.uint8, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    pulses = list(pulses)
    offs = [arrival_offsets(p.dm, nchan, f_top, foff, tsamp) for p in pulses]
    for r0 in range(0, nchan, rows_per_step):
        r1 = min(nchan, r0 + rows_per_step)
        x = torch.randn((r1 - r0, nsamp), generator=g, device=device, dtype=torch.float32)
        x.mul_(sigma).add_(mean)
        for p, off in zip(pulses, offs):
            sd = p.fwhm / _FWHM_PER_SIGMA
            rows, cols, vals = [], [], []
            for c in range(r0, r1):
                centre = p.t0 + off[c]
                lo = max(0, int(math.floor(centre - 6.0 * sd)) - 1)
                hi = min(nsamp, int(math.ceil(centre + 6.0 * sd)) + 2)
                if lo >= hi:
                    continue
                t = np.arange(lo, hi, dtype=np.float64)
                rows.append(np.full(hi - lo, c - r0))
                cols.append(t.astype(np.int64))
                vals.append((p.amp * np.exp(-0.5 * ((t - centre) / sd) ** 2)).astype(np.float32))
            if rows:
                ri = torch.from_numpy(np.concatenate(rows)).to(device)
                ci = torch.from_numpy(np.concatenate(cols)).to(device)
                vi = torch.from_numpy(np.concatenate(vals)).to(device)
                x.index_put_((ri, ci), vi, accumulate=True)
        torch.round(x, out=x)
        x.clamp_(0.0, 255.0)
        out[r0:r1, :nsamp] = x.to(torch.uint8)
        del x
    return out
