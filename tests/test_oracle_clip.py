"""Pins for the oracle's outlier-clipped statistics (CPU only): an independent loop over
Python integers and fractions, a closed form, reduction to the plain statistics, and
chunk invariance of a clipped search."""

import math

import numpy as np
import pytest

import oracle
from oracle.sps import block_norms, clipped_moments


def _loop_clip(vals, c, iters):
    """Plain loop: exact moments as integers, mu and sigma in float64 with the stated
    rounding points, the keep test in float64."""
    kept = [int(v) for v in vals]
    cf = float(np.float32(c))
    for _ in range(iters):
        n, a, b = len(kept), sum(kept), sum(v * v for v in kept)
        mu = a / n
        sigma = math.sqrt(float(n * b - a * a) / float(n * n))
        nxt = [int(v) for v in vals if abs(float(v) - mu) <= cf * sigma]
        if not nxt:
            break
        kept = nxt
    return len(kept), sum(kept), sum(v * v for v in kept)


@pytest.mark.parametrize("seed", range(6))
def test_clipped_moments_loop(seed):
    rng = np.random.default_rng(seed)
    rows = rng.integers(900, 1100, (3, 300)).astype(np.int64)
    for r in range(3):                                   # a few outliers per row
        rows[r, rng.integers(0, 300, 4)] = rng.integers(3000, 9000, 4)
    c, iters = [2.5, 3.0, 1.0][seed % 3], 1 + seed % 3
    n, s1, s2 = clipped_moments(rows, c, iters)
    for r in range(3):
        assert (n[r], s1[r], s2[r]) == _loop_clip(rows[r], c, iters)
        assert n[r] < 300                                # the outliers went


def test_clip_closed_form():
    """Alternating v, v+2 (mu v+1, sigma 1) plus one far outlier: one iteration at 3 sigma
    drops exactly the outlier, so the clipped mu and sigma are v+1 and 1."""
    v, n = 1000, 1000
    row = np.array([v, v + 2] * (n // 2) + [v + 100000], dtype=np.int64)[None, :]
    nn, s1, s2 = clipped_moments(row, 3.0, 1)
    assert nn == [n] and s1 == [n * (v + 1)] and s2 == [(n // 2) * (v * v + (v + 2) ** 2)]
    wmu, r = block_norms(nn, s1, s2, [1, 4])
    assert wmu[0, 0] == v + 1 and wmu[0, 1] == 4 * (v + 1)
    assert r[0, 0] == 1.0 and r[0, 1] == 0.5


def test_clip_off_is_plain(tiny, tiny_oracle):
    w, x = tiny
    for c, it in ((0.0, 3), (3.0, 0)):
        r = oracle.run(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"],
                       w["stat_block"], clip_sigma=c, clip_iters=it)
        assert r["candidates"] == tiny_oracle["candidates"]


def test_clip_raises_the_pulse_and_keeps_chunk_invariance(tiny, tiny_oracle):
    w, x = tiny
    args = (x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"])
    clipped = oracle.run(*args, 8192, clip_sigma=3.0, clip_iters=2)
    plain = oracle.run(*args, 8192)
    top_c = max(clipped["candidates"], key=lambda c: c[3])
    top_p = max(plain["candidates"], key=lambda c: c[3])
    assert top_c[:2] == top_p[:2] and top_c[3] >= top_p[3]   # the pulse no longer inflates sigma
    chunked = oracle.run_chunked(*args, 16384, 8192, clip_sigma=3.0, clip_iters=2)
    assert chunked == clipped["candidates"]


def test_clip_empty_keep_stops():
    """Two values 1 and 2 at c = 0.5: |v - 1.5| = 0.5 > 0.25, nothing would be kept, so the
    unclipped moments stay."""
    row = np.array([[1, 2] * 10], dtype=np.int64)
    assert clipped_moments(row, 0.5, 3) == ([20], [30], [50])
