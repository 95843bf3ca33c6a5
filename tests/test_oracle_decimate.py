"""Pins for the oracle's per-range time decimation (CPU only): brute force, exact
rational shifts, the decimate/dedisperse composition on pair-constant input, reduction to
the plain oracle, and recovery of an injected pulse in a decimated range."""

from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth.dmplan import dm_plan
from synth.filterbank import Pulse, make_filterbank


def _avg_loop(row):
    return [(int(row[2 * j]) + int(row[2 * j + 1]) + 1) // 2 for j in range(len(row) // 2)]


@pytest.mark.parametrize("n", [1, 2, 7, 64, 101])
def test_decimate2_bruteforce(n):
    rng = np.random.default_rng(n)
    x = rng.integers(0, 256, (3, n), dtype=np.uint8)
    got = oracle.decimate2(x)
    assert got.dtype == np.uint8 and got.shape == (3, n // 2)
    for c in range(3):
        assert list(got[c]) == _avg_loop(x[c])


def test_decimate_closed_forms():
    # half rounds up; equal pairs are kept; 255 pairs do not overflow
    x = np.array([[0, 1, 1, 2, 7, 7, 255, 255, 254, 255]], dtype=np.uint8)
    assert list(oracle.decimate2(x)[0]) == [1, 2, 7, 255, 255]
    # f = 4 halves twice: ((0+1+1)>>1 + (1+1+1)>>1 + 1) >> 1 = (1 + 1 + 1) >> 1 = 1
    assert list(oracle.decimate(np.array([[0, 1, 1, 1]], dtype=np.uint8), 4)[0]) == [1]
    # ... which differs from the rounded mean of the four samples, (0+1+1+1)/4 -> 1 here,
    # but e.g. [0, 1, 0, 1]: halvings give (1, 1) -> 1, the rounded mean 0.5 -> 1 as well;
    # [0, 0, 0, 1]: halvings (0, 1) -> 1, the mean 0.25 -> 0: each halving rounds
    assert list(oracle.decimate(np.array([[0, 0, 0, 1]], dtype=np.uint8), 4)[0]) == [1]
    with pytest.raises(ValueError):
        oracle.decimate(x, 3)


def _exact_shift(dm, c, f_top, foff, tsamp):
    K = Fraction(4.148808e3)
    fc = Fraction(f_top) - c * Fraction(foff)
    x = K * Fraction(dm) * (1 / (fc * fc) - 1 / (Fraction(f_top) ** 2)) / Fraction(tsamp) + Fraction(1, 2)
    return x.numerator // x.denominator


def test_range_shifts_exact_rational():
    dms = dm_plan(700)
    first, factor = [0, 512, 600], [1, 2, 4]
    plans = oracle.range_plans(dms, 64, 1 << 16, 1450.0, 300.0 / 64, 64e-6, [1, 2, 4], 32768, first, factor)
    rng = np.random.default_rng(3)
    for rp in plans:
        for _ in range(60):
            i = int(rng.integers(0, rp["hi"] - rp["lo"]))
            c = int(rng.integers(0, 64))
            want = _exact_shift(float(dms[rp["lo"] + i]), c, 1450.0, 300.0 / 64, rp["f"] * 64e-6)
            assert int(rp["shifts"][i, c]) == want
        assert rp["n"] == (1 << 16) // rp["f"] and rp["block"] == 32768 // rp["f"]


def test_decimated_dedispersion_composition():
    """Pair-constant input and a shift table that is exactly twice a half-resolution one:
    dedispersing the decimated input equals the full-resolution result at even samples."""
    rng = np.random.default_rng(5)
    nchan, n2 = 6, 300
    half = rng.integers(0, 256, (nchan, n2), dtype=np.uint8)
    x = np.repeat(half, 2, axis=1)                         # x[2j] == x[2j+1]
    s2 = np.sort(rng.integers(0, 25, (4, nchan)), axis=1)
    s1 = 2 * s2
    D1 = oracle.dedisperse(x, s1)
    D2 = oracle.dedisperse(oracle.decimate2(x), s2)
    assert np.array_equal(oracle.decimate2(x), half)
    assert np.array_equal(D1[:, 0::2][:, :D2.shape[1]], D2)


def test_single_range_factor_one_is_the_plain_oracle(tiny, tiny_oracle):
    w, x = tiny
    r = oracle.run_ranges(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"],
                          w["threshold"], w["stat_block"], [0], [1])
    assert r["candidates"] == tiny_oracle["candidates"]


def test_two_ranges_factor_one_match_plain_away_from_the_edge(tiny):
    """Splitting the trials changes only the peak test at the range edge (no neighbour
    across it) and each range's own maxshift, so its own T and its last, partial stat
    block. Over the stat blocks that are complete in both runs, trials away from the
    edge have the plain oracle's candidates exactly."""
    w, x = tiny
    B = 8192
    plain = oracle.run(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"], B)
    r = oracle.run_ranges(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"],
                          w["threshold"], B, [0, 60], [1, 1])
    full = plain["sizes"]["n_start"] // B * B          # starts in blocks complete in both runs
    edge = {59, 60}
    got = [c for c in r["candidates"] if c[0] not in edge and c[1] < full - 1]
    want = [c for c in plain["candidates"] if c[0] not in edge and c[1] < full - 1]
    assert got == want and len(want) > 10
    got_e = {c[:3] for c in r["candidates"] if c[0] in edge and c[1] < full - 1}
    want_e = {c[:3] for c in plain["candidates"] if c[0] in edge and c[1] < full - 1}
    assert want_e <= got_e            # removing neighbours can only add peaks


def test_pulse_recovered_in_a_decimated_range():
    nchan, nsamp, f_top, foff, tsamp = 64, 1 << 16, 1450.0, 300.0 / 64, 64e-6
    dms = np.arange(0, 400, 2.0)
    pulse = Pulse(dm=301.0, t0=30000.0, fwhm=12.0, amp=40.0)
    x = make_filterbank(nchan, nsamp, f_top, foff, tsamp, [pulse], seed=9)
    r = oracle.run_ranges(x, nsamp, f_top, foff, tsamp, dms, [1, 2, 4, 8], 6.0, 8192, [0, 100], [1, 4])
    top = max(r["candidates"], key=lambda c: c[3])
    assert abs(dms[top[0]] - 301.0) <= 4.0
    assert top[0] >= 100                                  # found in the decimated range
    assert top[1] % 4 == 0 and top[2] % 4 == 0            # starts and widths in input samples
    assert abs(top[1] + top[2] / 2 - 30000) <= 4 * 8


def test_survey_ranges_keep_the_bottom_step_near_one_sample():
    """With factor 2^r on the survey plan's r-th range, the bottom channel's shift grows by
    about one sample of the range's resolution per trial (the reason for the factors)."""
    dms = dm_plan(3000)
    first, factor = [0, 512, 1024, 1536, 2048, 2432], [1, 2, 4, 8, 16, 32]
    plans = oracle.range_plans(dms, 4096, 1 << 20, 1450.0, 300.0 / 4096, 64e-6, [1], 32768, first, factor)
    for rp in plans:
        step = np.diff(rp["shifts"][:, -1]).mean()
        assert 0.9 <= step <= 1.3, (rp["lo"], step)


def test_range_errors():
    with pytest.raises(ValueError):
        oracle.range_plans(np.arange(10.0), 4, 1000, 1400.0, 1.0, 1e-3, [1], 256, [1, 5], [1, 2])
    with pytest.raises(ValueError):
        oracle.range_plans(np.arange(10.0), 4, 1000, 1400.0, 1.0, 1e-3, [1], 256, [0, 5], [2, 1])
    with pytest.raises(ValueError):
        oracle.range_plans(np.arange(10.0), 4, 1000, 1400.0, 1.0, 1e-3, [1], 256, [0, 5], [1, 3])
