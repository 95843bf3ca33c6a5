"""Pins for the oracle's friends-of-friends clustering (CPU only): closed-form chains at
and beyond the radii, the peak tie rule, beams kept apart, and invariance under input
order."""

import random

import oracle


def test_chain_at_the_radius_is_one_cluster():
    c = [(5, 100 + 7 * k, 1, 6.0 + k) for k in range(6)]
    out = oracle.cluster(c, 0, 7)
    assert len(out) == 1 and out[0]["members"] == 6
    assert out[0]["peak"] == c[-1] and (out[0]["t_lo"], out[0]["t_hi"]) == (100, 135)
    assert len(oracle.cluster(c, 0, 6)) == 6                 # one less: all apart


def test_diagonal_across_trials():
    c = [(10 + 2 * k, 50 + 3 * k, 2, 7.0) for k in range(5)]
    out = oracle.cluster(c, 2, 3)
    assert len(out) == 1 and (out[0]["dm_lo"], out[0]["dm_hi"]) == (10, 18)
    assert len(oracle.cluster(c, 1, 3)) == 5
    assert len(oracle.cluster(c, 2, 2)) == 5


def test_transitive_link_through_a_middle_member():
    # a and c are 2 apart in t (radius 1) and linked only through b
    c = [(0, 0, 1, 6.0), (1, 1, 1, 6.5), (0, 2, 1, 6.2)]
    out = oracle.cluster(c, 1, 1)
    assert len(out) == 1 and out[0]["members"] == 3 and out[0]["peak"] == c[1]


def test_peak_tie_takes_the_smallest_trial_then_start():
    c = [(3, 10, 1, 9.0), (2, 12, 1, 9.0), (2, 11, 4, 9.0), (4, 9, 1, 8.0)]
    out = oracle.cluster(c, 2, 5)
    assert len(out) == 1 and out[0]["peak"] == (2, 11, 4, 9.0)


def test_beams_are_kept_apart():
    c = [(0, 0, 1, 6.0), (0, 0, 1, 7.0)]
    assert len(oracle.cluster(c, 5, 5, beams=[0, 1])) == 2
    assert len(oracle.cluster(c, 5, 5, beams=[1, 1])) == 1


def test_order_invariance_and_member_total():
    rng = random.Random(4)
    c = [(rng.randrange(0, 40), rng.randrange(0, 400), 1, rng.choice([6.0, 6.5, 7.0, 8.0])) for _ in range(150)]
    a = oracle.cluster(c, 2, 9)
    d = c[:]
    rng.shuffle(d)
    assert oracle.cluster(d, 2, 9) == a
    assert sum(x["members"] for x in a) == len(c)
    assert len(a) < len(c)
    # far apart in t, no link at all: one cluster per candidate
    far = [(k % 3, 1000 * k, 1, 6.0) for k in range(20)]
    assert len(oracle.cluster(far, 5, 999)) == 20
