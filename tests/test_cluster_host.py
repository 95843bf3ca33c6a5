"""aa_cluster (host code in the library) against the oracle's friends-of-friends
clustering: random candidate sets, several beams, radii from none to wide, and the
candidate list of the small workload."""

import numpy as np
import pytest

import oracle


def _arr(cands, beams=None):
    from paper_2101_00941_amd import CANDIDATE_DTYPE
    a = np.zeros(len(cands), dtype=CANDIDATE_DTYPE)
    for i, (d, t, w, s) in enumerate(cands):
        a[i] = (d, w, t, s, 0 if beams is None else beams[i])
    return a


def _lib_clusters(cands, rd, rt, beams=None):
    from paper_2101_00941_amd import cluster
    out = cluster(_arr(cands, beams), rd, rt)
    return [dict(beam=int(c["peak"]["beam"]), peak=(int(c["peak"]["dm_idx"]), int(c["peak"]["t"]),
                 int(c["peak"]["width"]), float(c["peak"]["snr"])), members=int(c["members"]),
                 dm_lo=int(c["dm_lo"]), dm_hi=int(c["dm_hi"]), t_lo=int(c["t_lo"]), t_hi=int(c["t_hi"]))
            for c in out]


@pytest.mark.parametrize("seed", range(8))
def test_random_sets_match_oracle(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    cands = [(int(rng.integers(0, 60)), int(rng.integers(0, 2000)), int(rng.choice([1, 2, 4])),
              float(np.float32(rng.choice([6.0, 6.25, 7.5, 9.0, 12.0])))) for _ in range(n)]
    beams = [int(b) for b in rng.integers(0, 3, n)]
    for rd, rt in ((0, 0), (1, 10), (3, 50), (10, 400)):
        assert _lib_clusters(cands, rd, rt, beams) == oracle.cluster(cands, rd, rt, beams)


def test_small_workload_candidates(tiny_oracle):
    cands = [(d, t, w, float(np.float32(s))) for d, t, w, s in tiny_oracle["candidates"]]
    for rd, rt in ((2, 16), (5, 64)):
        got = _lib_clusters(cands, rd, rt)
        assert got == oracle.cluster(cands, rd, rt)
    # the injected pulse (trial 50) is the peak of the strongest cluster, which also holds
    # its neighbours in trial; the off-DM responses of the pulse form clusters of their own
    top = max(oracle.cluster(cands, 5, 64), key=lambda c: c["peak"][3])
    assert top["peak"][0] == 50 and top["dm_lo"] < 50 < top["dm_hi"] and top["members"] > 1


def test_cluster_errors_and_empty():
    from paper_2101_00941_amd import AAError, cluster
    assert len(cluster(_arr([]), 1, 1)) == 0
    with pytest.raises(AAError):
        cluster(_arr([(0, 0, 1, 6.0)]), -1, 1)
