"""GPU test of aa_single_pulse_noalloc (the search for callers that cannot allocate):
through the C ABI, its candidates, counts and best-S/N plane must equal those of
aa_single_pulse with a work buffer, bit for bit, on two calls in a row on one GPU, the
second with a smaller input (fewer trials, fewer starts, another plan), so the second
call runs on scratch that still holds the first call's contents. Oversized requests
must be refused."""

import numpy as np
import pytest

from synth.filterbank import Pulse, make_filterbank
from tests.gpu_util import say, to_device

pytestmark = pytest.mark.gpu


def _case(nchan, nsamp, ndm, seed, stat_block):
    from paper_2101_00941_amd import Plan
    dms = np.arange(ndm) * 1.0
    x = make_filterbank(nchan, nsamp, 1500.0, 0.78125, 64e-6, [Pulse(float(dms[ndm // 2]), nsamp * 0.6, 4.0, 48.0)],
                       seed=seed)
    plan = Plan(nchan, nsamp, 1500.0, 0.78125, 64e-6, dms, [1, 2, 4, 8, 16, 32], 6.0, stat_block)
    D = plan.dedisperse(to_device(x, nsamp), n_in=nsamp)
    return plan, D


def _both(plan, D, t_begin=0, t_end=None):
    import torch
    from paper_2101_00941_amd import candidates_as_tuples, candidates_to_numpy
    T = plan.info["n_start"]
    t_end = T if t_end is None else t_end
    cap = 4096
    c1, n1, b1 = plan.single_pulse(D, t_begin=t_begin, t_end=t_end, cap=cap, want_best=True)
    cand = torch.full((cap * 24,), 0xAB, dtype=torch.uint8, device="cuda")
    count = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    best = torch.full_like(b1, -1.0)
    plan.single_pulse_noalloc(D, cand, count, t_begin=t_begin, t_end=t_end, cap=cap, best=best)
    torch.cuda.synchronize()
    a = candidates_as_tuples(candidates_to_numpy(c1, n1, cap))
    b = candidates_as_tuples(candidates_to_numpy(cand, count, cap))
    assert int(n1.item()) == int(count.item())
    assert a == b                                   # same kernels: identical lists and S/N bits
    n = t_end - t_begin
    assert torch.equal(b1[:, :n], best[:, :n])
    return a


def test_noalloc_matches_work_buffer_entry_point_twice():
    big, Db = _case(128, 200_000, 100, 61, 32768)
    small, Ds = _case(64, 60_000, 37, 62, 8192)
    say("noalloc: large call")
    a = _both(big, Db)
    assert len(a) > 0
    say("noalloc: smaller call on the same scratch")
    b = _both(small, Ds)
    assert len(b) > 0
    say("noalloc: a block-aligned sub-range of the large plane")
    _both(big, Db, t_begin=32768, t_end=100_000)


def test_noalloc_refuses_oversized_search():
    import torch
    from paper_2101_00941_amd import AAError, Plan
    # 8192 trials x 2^17 starts need 128 MiB of mask scratch, beyond the fixed array
    nsamp = (1 << 17) + 64
    plan = Plan(16, nsamp, 1500.0, 0.78125, 64e-6, np.arange(8192) * 0.001, [1, 2, 4], 6.0)
    T = plan.info["n_start"]
    assert plan.work_bytes(T) > 64 << 20
    D = torch.zeros((8192, plan.info["out_pitch"]), dtype=torch.int32, device="cuda")
    cand = torch.empty(24 * 16, dtype=torch.uint8, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(AAError) as e:
        plan.single_pulse_noalloc(D, cand, count, cap=16)
    assert e.value.code == -1 and "scratch" in str(e.value)
    # a block-aligned part of the same search fits, and runs
    plan.single_pulse_noalloc(D, cand, count, t_begin=0, t_end=32768, t_total=T, cap=16)
    torch.cuda.synchronize()
    assert int(count.item()) == 0      # a constant plane has sigma 0: S/N 0, no candidates
