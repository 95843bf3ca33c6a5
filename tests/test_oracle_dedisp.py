"""Pins for the oracle's dedispersion (CPU only): brute force by hand, closed forms,
invariants."""

import numpy as np
import pytest

import oracle


def _bruteforce(x, shifts, n_out):
    """Literal definition, one Python loop per index."""
    ndm, nchan = shifts.shape
    out = [[0] * n_out for _ in range(ndm)]
    for d in range(ndm):
        for t in range(n_out):
            acc = 0
            for c in range(nchan):
                acc += int(x[c][t + int(shifts[d][c])])
            out[d][t] = acc
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_bruteforce_tiny_random(seed):
    rng = np.random.default_rng(seed)
    nchan, nsamp, ndm = int(rng.integers(1, 9)), int(rng.integers(40, 129)), int(rng.integers(1, 7))
    x = rng.integers(0, 256, (nchan, nsamp), dtype=np.uint8)
    # random monotone shift rows (any table works for the definition)
    shifts = np.sort(rng.integers(0, 20, (ndm, nchan)), axis=1)
    n_out = nsamp - int(shifts.max())
    got = oracle.dedisperse(x, shifts, nsamp)
    assert got.shape == (ndm, n_out)
    assert np.array_equal(got, _bruteforce(x, shifts, n_out))


def test_bruteforce_real_plan():
    rng = np.random.default_rng(11)
    nchan, nsamp = 8, 200
    s = oracle.shift_table(np.array([0.0, 30.0, 61.5, 120.0]), nchan, 1400.0, 12.5, 1e-3)
    x = rng.integers(0, 256, (nchan, nsamp), dtype=np.uint8)
    n_out = nsamp - int(s.max())
    assert np.array_equal(oracle.dedisperse(x, s, nsamp), _bruteforce(x, s, n_out))


def test_dm0_is_channel_sum(tiny):
    w, x = tiny
    s = oracle.shift_table(w["dms"][:3], w["nchan"], w["f_top"], w["foff"], w["tsamp"])
    D = oracle.dedisperse(x, s, w["nsamp"], maxshift=418)
    assert np.array_equal(D[0], x.astype(np.int64).sum(axis=0)[:w["nsamp"] - 418])


def test_single_channel_is_identity():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 256, (1, 500), dtype=np.uint8)
    s = oracle.shift_table(np.array([0.0, 100.0, 500.0]), 1, 1400.0, 1.0, 64e-6)
    assert (s == 0).all()
    D = oracle.dedisperse(x, s, 500)
    assert np.array_equal(D, np.repeat(x.astype(np.int64), 3, axis=0))


def test_impulse_response():
    # one unit sample at (c, t) lands at t - s[d][c] in every row d
    nchan, nsamp = 16, 300
    s = oracle.shift_table(np.array([0.0, 3.0, 7.25, 20.0]), nchan, 1500.0, 2.0, 64e-6)
    m = int(s.max())
    for c, t in [(0, 150), (15, 299), (7, 120)]:
        x = np.zeros((nchan, nsamp), np.uint8)
        x[c, t] = 1
        D = oracle.dedisperse(x, s, nsamp)
        for d in range(4):
            want = np.zeros(nsamp - m, np.int64)
            if 0 <= t - s[d, c] < nsamp - m:
                want[t - s[d, c]] = 1
            assert np.array_equal(D[d], want), (c, t, d)


def test_linearity():
    rng = np.random.default_rng(9)
    s = oracle.shift_table(np.linspace(0, 80, 9), 32, 1500.0, 1.5, 64e-6)
    a = rng.integers(0, 128, (32, 1000), dtype=np.uint8)
    b = rng.integers(0, 128, (32, 1000), dtype=np.uint8)
    assert np.array_equal(oracle.dedisperse(a + b, s, 1000),
                          oracle.dedisperse(a, s, 1000) + oracle.dedisperse(b, s, 1000))


def test_rows_subset_matches_full():
    rng = np.random.default_rng(2)
    s = oracle.shift_table(np.linspace(0, 40, 12), 24, 1500.0, 1.5, 64e-6)
    x = rng.integers(0, 256, (24, 700), dtype=np.uint8)
    full = oracle.dedisperse(x, s, 700)
    assert np.array_equal(oracle.dedisperse_rows(x, s, [11, 0, 5], 700), full[[11, 0, 5]])
