"""Pins for the oracle's decimated boxcar hierarchy (CPU only): closed-form strides, the
defining equality with boxcars on decimated planes, a brute-force loop, reduction to the
plain search, and the bound against the plain best plane."""

import math

import numpy as np
import pytest

import oracle
from oracle.sps import best_plane, block_moments, block_norms, boxcar_strides


def test_stride_closed_forms():
    p2 = [1, 2, 4, 8, 16, 32, 64, 128, 256]
    assert boxcar_strides(p2, 32) == [1, 1, 1, 1, 1, 1, 2, 4, 8]
    assert boxcar_strides(p2, 0) == [1] * 9
    assert boxcar_strides(p2, 1) == p2
    assert boxcar_strides([50, 65, 96], 32) == [2, 4, 4]


def _plane(seed, rows=3, n=600):
    rng = np.random.default_rng(seed)
    D = rng.integers(1000, 1100, (rows, n)).astype(np.int64)
    D[:, 300:340] += 60                      # a wide bump
    return D


def test_strided_widths_are_boxcars_of_decimated_planes():
    """A width-w boxcar at a start that is a multiple of its stride s equals the width-w/s
    boxcar of the plane decimated by s (sums of s adjacent samples), at start t / s."""
    D = _plane(1)
    widths, w0 = [1, 2, 4, 8, 16, 32], 4
    strides = boxcar_strides(widths, w0)
    n, s1, s2 = block_moments(D)
    wmu, r = block_norms(n, s1, s2, widths)
    prefix = np.zeros((D.shape[0], D.shape[1] + 1), dtype=np.int64)
    np.cumsum(D, axis=1, out=prefix[:, 1:])
    T = D.shape[1] - max(widths) + 1
    best, widx = best_plane(prefix, 0, 0, T, widths, wmu, r, strides)
    for i in range(D.shape[0]):
        for t in range(0, T, 7):
            vals = []
            for k, (w, s) in enumerate(zip(widths, strides)):
                if t % s:
                    continue
                Ds = D[i, : (D.shape[1] // s) * s].reshape(-1, s).sum(axis=1)   # decimated by s
                ssum = int(Ds[t // s: t // s + w // s].sum())
                vals.append(((float(ssum) - wmu[i, k]) * r[i, k], k))
            v = max(x for x, _ in vals)
            assert best[i, t] == v
            assert widx[i, t] == min(k for x, k in vals if x == v)


def test_bruteforce_loop_tiny():
    D = _plane(2, rows=2, n=120)
    widths, w0 = [1, 3, 8, 20], 3
    strides = boxcar_strides(widths, w0)
    assert strides == [1, 1, 4, 8]
    n, s1, s2 = block_moments(D)
    wmu, r = block_norms(n, s1, s2, widths)
    prefix = np.zeros((2, 121), dtype=np.int64)
    np.cumsum(D, axis=1, out=prefix[:, 1:])
    T = 120 - 20 + 1
    best, _ = best_plane(prefix, 0, 0, T, widths, wmu, r, strides)
    for i in range(2):
        mu = s1[i] / n
        sigma = math.sqrt(float(n * s2[i] - s1[i] * s1[i]) / float(n * n))
        for t in range(T):
            v = -math.inf
            for w, s in zip(widths, strides):
                if t % s == 0:
                    ssum = sum(int(D[i, t + j]) for j in range(w))
                    v = max(v, (float(ssum) - float(w) * mu) * (1.0 / (sigma * math.sqrt(float(w)))))
            assert best[i, t] == v


def test_hierarchy_off_or_wide_is_plain(tiny, tiny_oracle):
    w, x = tiny
    for w0 in (0, 32, 64):
        r = oracle.run(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"],
                       w["stat_block"], boxcar_full_width=w0)
        assert r["candidates"] == tiny_oracle["candidates"]


def test_hierarchy_bounds_and_pulse(tiny, tiny_oracle):
    w, x = tiny
    r = oracle.run(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"],
                   w["stat_block"], want_best=True, boxcar_full_width=4)
    plain = tiny_oracle["best"]
    assert (r["best"] <= plain).all()
    # at starts that are multiples of every stride (8 for widths 1..32 at w0 = 4) nothing changes
    assert np.array_equal(r["best"][:, ::8], plain[:, ::8])
    top = max(r["candidates"], key=lambda c: c[3])
    assert top[0] == 50
    with pytest.raises(ValueError):
        oracle.run(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], [4, 8], w["threshold"],
                   w["stat_block"], boxcar_full_width=2)


def test_hierarchy_chunk_invariance(tiny):
    w, x = tiny
    args = (x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"], w["threshold"])
    whole = oracle.run(*args, 4096, boxcar_full_width=8)["candidates"]
    assert oracle.run_chunked(*args, 8192, 4096, boxcar_full_width=8) == whole
