"""Helpers for the GPU parity tests: upload a numpy filterbank and run the HIP path
through the C ABI (via the ctypes binding)."""

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_device(x: np.ndarray, nsamp: int, pitch: int | None = None, fill: int = 255):
    """uint8 [nchan, pitch] CUDA tensor. Columns past nsamp hold `fill`, to catch reads
    past the valid samples."""
    import torch
    nchan = x.shape[0]
    pitch = pitch or (nsamp + 255) // 256 * 256
    host = np.full((nchan, pitch), fill, dtype=np.uint8)
    host[:, :nsamp] = x[:, :nsamp]
    return torch.from_numpy(host).cuda()


def run_gpu(plan, x: np.ndarray, nsamp: int, cap: int = 1 << 16, want_best: bool = True, pitch=None):
    """Dedisperse the whole input, then search every start. Returns numpy results."""
    import torch
    from paper_2101_00941_amd import candidates_as_tuples, candidates_to_numpy
    xd = to_device(x, nsamp, pitch)
    D = plan.dedisperse(xd, n_in=nsamp)
    cand, count, best = plan.single_pulse(D, cap=cap, want_best=want_best)
    torch.cuda.synchronize()
    n_dd, T = plan.info["n_dd"], plan.info["n_start"]
    cands = candidates_as_tuples(candidates_to_numpy(cand, count, cap))
    return dict(D=D[:, :n_dd].cpu().numpy().astype(np.int64), candidates=cands, count=int(count.item()),
                best=None if best is None else best[:, :T].cpu().numpy())


def assert_candidates_equal(got, want, rtol=1e-5):
    """Identical (dm_idx, t, width) lists. S/N within rtol relative."""
    assert [(d, t, w) for d, t, w, _ in got] == [(d, t, w) for d, t, w, _ in want]
    for g, h in zip(got, want):
        assert abs(g[3] - h[3]) <= rtol * max(1.0, abs(h[3])), (g, h)
