"""Regression pin: the oracle still reproduces the stored tiny-workload candidate list."""

import os

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_tiny_candidates_unchanged(tiny_oracle):
    rows = []
    with open(os.path.join(HERE, "tiny_candidates.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            d, t, w, snr = line.split()
            rows.append((int(d), int(t), int(w), float(snr)))
    assert rows == tiny_oracle["candidates"]
