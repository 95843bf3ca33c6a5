"""DM-trial lists for the survey-size workloads.

The survey workload asks for a DM plan whose step doubles from one range to the
next. The plan used here has six ranges:

  range   step     trials    first DM
  1       1/16     512       0
  2       1/8      512       32
  3       1/4      512       96
  4       1/2      512       224
  5       1        384       480
  6       2        rest      864

Every value is an exact binary fraction, so the float64 list is exact. Plans
shorter than 2432 trials stop partway through a range. 3000 trials end at
DM 1998 and 4096 trials end at DM 4190.
"""

import numpy as np

_RANGES = ((1.0 / 16, 512), (1.0 / 8, 512), (1.0 / 4, 512), (1.0 / 2, 512), (1.0, 384), (2.0, None))


def dm_plan(n: int) -> np.ndarray:
    """Return `n` ascending DM trials (pc cm^-3, float64) of the doubling-step plan."""
    if n < 1:
        raise ValueError("a DM plan needs at least one trial")
    out = []
    start = 0.0
    for step, count in _RANGES:
        take = n - len(out) if count is None else min(count, n - len(out))
        out.extend(start + step * i for i in range(take))
        if count is not None:
            start += step * count
        if len(out) == n:
            break
    return np.asarray(out, dtype=np.float64)


def uniform_plan(n: int, step: float = 1.0, first: float = 0.0) -> np.ndarray:
    """`n` trials first, first+step, ... (the small workload uses DM 0..99 step 1)."""
    return first + step * np.arange(n, dtype=np.float64)
