"""MI355X (gfx950) brute-force dedispersion and single-pulse search.

The HIP library `libaa_mi355x.so` (built from csrc/) does all the computation
behind the C ABI in include/aa.h. This package is a thin ctypes binding with the
same names. See api.Plan.
"""

from ._native import AAError, CANDIDATE_DTYPE, LIB_PATH, lib
from .api import Pipeline, Plan, RangePlan, batch_run, candidates_as_tuples, candidates_to_numpy, cluster, decimate2

__all__ = ["AAError", "CANDIDATE_DTYPE", "LIB_PATH", "lib", "Pipeline", "Plan", "RangePlan", "batch_run",
           "candidates_as_tuples", "candidates_to_numpy", "cluster", "decimate2"]
