"""Pins for the oracle's shift table (CPU only).

The shift table is checked against things other than its own float64 formula:
* exact rational arithmetic on the same float64 inputs, which checks the rounding
  and the operation order;
* invariants that the dispersion law fixes: shift 0 at the top channel, monotone in
  channel and DM, linear in DM, and the f^-2 ratio between channels;
* recovery of a pulse placed by the independent signal model (see test_oracle_sps).
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import dm_plan
from synth.workloads import workload


def _exact_shift(dm, c, f_top, foff, tsamp):
    K = Fraction(oracle.K_DM)
    ft = Fraction(f_top)
    fc = ft - c * Fraction(foff)
    x = K * Fraction(dm) * (1 / (fc * fc) - 1 / (ft * ft)) / Fraction(tsamp)
    fl = x.numerator // x.denominator
    frac = x - fl
    return (fl + 1 if frac >= Fraction(1, 2) else fl), abs(float(frac - Fraction(1, 2)))


@pytest.mark.parametrize("name", ["tiny_128ch_32k", "survey_4096ch_1M"])
def test_shift_table_matches_exact_rationals(name):
    w = workload(name)
    s = oracle.shift_table(w["dms"], w["nchan"], w["f_top"], w["foff"], w["tsamp"])
    rng = np.random.default_rng(7)
    if name == "tiny_128ch_32k":
        cells = [(d, c) for d in range(len(w["dms"])) for c in range(w["nchan"])]
    else:
        cells = [(int(d), int(c)) for d, c in zip(rng.integers(0, len(w["dms"]), 3000),
                                                 rng.integers(0, w["nchan"], 3000))]
        cells += [(len(w["dms"]) - 1, w["nchan"] - 1), (0, w["nchan"] - 1)]
    near_ties = []
    for d, c in cells:
        exact, dist = _exact_shift(w["dms"][d], c, w["f_top"], w["foff"], w["tsamp"])
        if dist < 1e-9:
            near_ties.append((d, c))
            continue
        assert s[d, c] == exact, (d, c)
    assert near_ties == []


def test_tiny_plan_values():
    w = workload("tiny_128ch_32k")
    s = oracle.shift_table(w["dms"], w["nchan"], w["f_top"], w["foff"], w["tsamp"])
    # 1400.78125 MHz bottom channel, DM 50: 13.52 ms of delay = 211.30 samples of 64 us
    assert s[50, 127] == 211 and s[1, 127] == 4 and s[50, 64] == 101
    sz = oracle.sizes(s, w["nsamp"], w["widths"], w["stat_block"])
    assert sz == dict(maxshift=418, n_dd=32350, n_start=32319, wmax=32, nblocks=1)


def test_survey_plan_sizes():
    w = workload("survey_4096ch_1M")
    assert w["dms"][-1] == 1998.0 and len(w["dms"]) == 3000
    s = oracle.shift_table(w["dms"], w["nchan"], w["f_top"], w["foff"], w["tsamp"])
    sz = oracle.sizes(s, w["nsamp"], w["widths"], w["stat_block"])
    assert sz["maxshift"] == 36321
    assert sz["n_dd"] == (1 << 20) - 36321 and sz["n_start"] == sz["n_dd"] - 255


def test_shift_invariants():
    dms = dm_plan(700)
    s = oracle.shift_table(dms, 512, 1450.0, 300.0 / 512, 64e-6)
    assert (s[:, 0] == 0).all()                       # top channel: no delay
    assert (np.diff(s, axis=1) >= 0).all()            # lower frequency, later arrival
    assert (np.diff(s, axis=0) >= 0).all()            # larger DM, larger delay
    assert (s[0] == 0).all()                          # DM 0
    # linear in DM: trial with twice the DM has twice the shift, up to rounding
    i, j = np.searchsorted(dms, 20.0), np.searchsorted(dms, 40.0)
    assert dms[i] * 2 == dms[j]
    assert np.abs(s[j] - 2 * s[i]).max() <= 1
    # f^-2 law between the bottom and the middle channel at a large DM
    f = 1450.0 - np.arange(512) * (300.0 / 512)
    ratio = (f[511] ** -2 - 1450.0 ** -2) / (f[256] ** -2 - 1450.0 ** -2)
    assert abs(s[-1, 511] / s[-1, 256] - ratio) < 2.0 / s[-1, 256]


def test_paper_setup_maxshift():
    # The paper's own run: 1400 MHz centre, 300 MHz, 4096 channels, 64 us, DM up to 3000.
    nchan = 4096
    foff = 300.0 / nchan
    f_top = 1400.0 + 150.0 - foff / 2
    s = oracle.shift_table(np.array([3000.0]), nchan, f_top, foff, 64e-6)
    # Continuous delay across the band: 4.148808 s * 3000 * (1250.0357^-2 - 1549.9634^-2) MHz^2
    f_lo = f_top - (nchan - 1) * foff
    approx = 4.148808e3 * 3000 * (f_lo ** -2 - f_top ** -2) / 64e-6
    assert abs(int(s.max()) - approx) <= 0.5
    assert 43000 < s.max() < 44000
