"""Pins for the oracle's single-pulse search (CPU only): closed forms, a library
z-score, brute-force boxcars and peaks, noise statistics, the injected pulse, and
chunk invariance."""

import math

import numpy as np
import pytest

import oracle
from synth.filterbank import Pulse, make_filterbank
from oracle.sps import best_plane, block_moments, block_norms, single_pulse


def test_constant_plus_impulse_closed_form():
    # A row that is c everywhere except c + h at one start t*. Over a block of n
    # starts: mu = c + h/n and sigma = h sqrt(n-1)/n. A window of width w that holds
    # t* then has S/N = (n - w) / (sqrt(n-1) sqrt(w)), whatever c and h are.
    n, c, h, ts = 1000, 5000, 77, 400
    widths = [1, 2, 4, 8]
    D = np.full((1, n + 16), c, dtype=np.int64)
    D[0, ts] += h
    _, best = single_pulse(D, 0, 0, n, n, widths, -1e9, stat_block=1024, want_best=True)
    assert abs(best[0, ts] - math.sqrt(n - 1)) < 1e-4          # w = 1 wins at t*
    assert abs(math.sqrt(999) - 31.6069612585582) < 1e-12
    # one start earlier: widths >= 2 hold t*, and the best of them is w = 2
    assert abs(best[0, ts - 1] - (n - 2) / (math.sqrt(n - 1) * math.sqrt(2))) < 1e-4
    # far from t*, every window misses it: S/N = -sqrt(w)/sqrt(n-1), best at w = 1
    assert abs(best[0, 100] - (-1 / math.sqrt(n - 1))) < 1e-6
    prefix = np.concatenate([[0], np.cumsum(D[0])])[None, :]
    nn, s1, s2 = block_moments(D[:, :n])
    wmu, r = block_norms(nn, s1, s2, [4])
    v, _ = best_plane(prefix, 0, ts - 3, ts + 1, [4], wmu, r)
    assert np.allclose(v[0], (n - 4) / (math.sqrt(n - 1) * 2.0), rtol=1e-12)


def test_width_one_is_library_zscore():
    rng = np.random.default_rng(3)
    D = rng.integers(1000, 5000, (3, 2100)).astype(np.int64)
    n = 2048
    nn, s1, s2 = block_moments(D[:, :n])
    wmu, r = block_norms(nn, s1, s2, [1])
    prefix = np.zeros((3, D.shape[1] + 1), np.int64)
    np.cumsum(D, axis=1, out=prefix[:, 1:])
    v, _ = best_plane(prefix, 0, 0, n, [1], wmu, r)
    z = (D[:, :n] - D[:, :n].mean(axis=1, keepdims=True)) / D[:, :n].std(axis=1, keepdims=True)
    assert np.allclose(v, z, rtol=1e-11, atol=1e-11)


def test_boxcar_sums_bruteforce():
    rng = np.random.default_rng(4)
    D = rng.integers(0, 1 << 20, (2, 300)).astype(np.int64)
    prefix = np.zeros((2, 301), np.int64)
    np.cumsum(D, axis=1, out=prefix[:, 1:])
    for w in [1, 3, 7, 64]:
        v, _ = best_plane(prefix, 0, 10, 200, [w], np.zeros((2, 1)), np.ones((2, 1)))
        for row in range(2):
            for t in range(10, 200):
                assert v[row, t - 10] == float(sum(int(a) for a in D[row, t:t + w]))


def _bruteforce_candidates(D, widths, thr, B, T):
    """Literal rule, written independently: numpy mean/std per (row, block), direct
    window sums, and an explicit loop over the 8 neighbours."""
    ndm = D.shape[0]

    def val(dd, t, b):
        seg = D[dd, b * B:min((b + 1) * B, T)].astype(np.float64)
        mu, sd = seg.mean(), seg.std()
        vals = [(float(D[dd, t:t + w].sum()) - w * mu) / (sd * math.sqrt(w)) for w in widths]
        k = int(np.argmax(vals))
        return vals[k], widths[k]

    out, margins = [], []
    for d in range(ndm):
        for t in range(T):
            b = t // B
            v, w = val(d, t, b)
            if v < thr:
                margins.append(thr - v)
                continue
            ok = True
            for dd in (d - 1, d, d + 1):
                for tt in (t - 1, t, t + 1):
                    if (dd, tt) == (d, t) or not (0 <= dd < ndm and 0 <= tt < T):
                        continue
                    u, _ = val(dd, tt, b)
                    if u != v:  # exact ties are broken by position, the same way on both sides
                        margins.append(abs(v - u))
                    earlier = dd < d or (dd == d and tt < t)
                    if (earlier and not v > u) or (not earlier and not v >= u):
                        ok = False
            if ok:
                out.append((d, t, w, v))
    return out, min(margins)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_peaks_bruteforce(seed):
    rng = np.random.default_rng(seed)
    ndm, T, B, widths = 5, 96, 32, [1, 2, 4]
    D = rng.integers(0, 5000, (ndm, T + 3)).astype(np.int64)
    D[rng.integers(0, ndm), rng.integers(0, T)] += 40000          # one clear peak
    want, margin = _bruteforce_candidates(D, widths, 1.5, B, T)
    assert margin > 1e-9
    got, _ = single_pulse(D, 0, 0, T, T, widths, 1.5, B)
    assert [(d, t, w) for d, t, w, _ in got] == [(d, t, w) for d, t, w, _ in want]
    for g, h in zip(got, want):
        assert abs(g[3] - h[3]) <= 1e-5 * abs(h[3])


def test_plateau_tie_break():
    # equal values: the first in row-major order is the only peak
    D = np.zeros((3, 40), np.int64)
    D[1, 20] = D[1, 21] = 100
    got, _ = single_pulse(D, 0, 0, 38, 38, [1], 1.0, 64)
    assert [(d, t) for d, t, _, _ in got] == [(1, 20)]


def test_constant_input_has_no_candidates():
    D = np.full((4, 500), 77, np.int64)
    got, best = single_pulse(D, 0, 0, 490, 490, [1, 2, 4], -5.0, 128, want_best=True)
    assert got == [] or all(c[3] == 0.0 for c in got)
    assert (best == 0).all()


def test_noise_exceedance_matches_gaussian_tail():
    rng = np.random.default_rng(12)
    D = rng.normal(1e5, 300.0, (4, 1 << 16)).round().astype(np.int64)
    _, best = single_pulse(D, 0, 0, (1 << 16) - 1, (1 << 16) - 1, [1], -1e9, 1 << 14, want_best=True)
    for thr in (1.0, 2.0, 3.0):
        q = 0.5 * math.erfc(thr / math.sqrt(2))
        frac = float((best >= thr).mean())
        n = best.size
        assert abs(frac - q) < 5 * math.sqrt(q * (1 - q) / n) + 1e-4, (thr, frac, q)


def test_injected_pulse_recovered(tiny_oracle, tiny):
    w, _ = tiny
    c = tiny_oracle["candidates"]
    d, t, wb, snr = max(c, key=lambda q: q[3])
    p = w["pulses"][0]
    assert d == 50 and w["dms"][d] == p.dm
    assert abs(t + (wb - 1) / 2 - p.t0) <= wb / 2 + 1
    assert snr > 30


def test_pulse_recovered_at_other_dms():
    # independent signal model at several DMs and arrival times, no noise clipping issues
    nchan, nsamp, f_top, foff, tsamp = 64, 6000, 1500.0, 2.0, 64e-6
    dms = np.arange(0, 120, 2.0)
    for dm, t0 in [(0.0, 1000.0), (37.0, 2500.5), (98.0, 3333.0)]:
        x = make_filterbank(nchan, nsamp, f_top, foff, tsamp, [Pulse(dm, t0, 3.0, 60.0)], seed=int(dm))
        r = oracle.run(x, nsamp, f_top, foff, tsamp, dms, [1, 2, 4, 8], 6.0, stat_block=2048)
        d, t, wb, _ = max(r["candidates"], key=lambda q: q[3])
        assert abs(dms[d] - dm) <= 2.0, (dm, dms[d])
        assert abs(t + (wb - 1) / 2 - t0) <= wb / 2 + 1, (dm, t, wb)


def test_chunked_equals_whole():
    nchan, nsamp, f_top, foff, tsamp = 32, 40000, 1500.0, 1.5, 64e-6
    dms = np.arange(0, 60, 1.0)
    pulses = [Pulse(30.0, 8191.0, 4.0, 90.0), Pulse(12.0, 16384.0, 2.0, 90.0), Pulse(55.0, 31000.0, 8.0, 70.0)]
    x = make_filterbank(nchan, nsamp, f_top, foff, tsamp, pulses, seed=8)
    widths = [1, 2, 4, 8, 16]
    whole = oracle.run(x, nsamp, f_top, foff, tsamp, dms, widths, 5.0, stat_block=4096)["candidates"]
    for chunk in (4096, 8192, 12288):
        assert oracle.run_chunked(x, nsamp, f_top, foff, tsamp, dms, widths, 5.0, chunk, 4096) == whole
    assert len(whole) > 3


def test_block_stats_are_per_block():
    # two blocks with different noise levels: each is normalised by its own sigma
    rng = np.random.default_rng(6)
    B = 4096
    D = np.concatenate([rng.normal(1e4, 10, B), rng.normal(1e4, 1000, B + 10)]).round().astype(np.int64)[None]
    _, best = single_pulse(D, 0, 0, 2 * B, 2 * B, [1], -1e9, B, want_best=True)
    assert 0.9 < best[0, :B].std() < 1.1 and 0.9 < best[0, B:].std() < 1.1
