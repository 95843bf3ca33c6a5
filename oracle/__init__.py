"""CPU oracle for brute-force incoherent dedispersion plus single-pulse search.

THIS PACKAGE IS TEST INFRASTRUCTURE. It is the plain, slow and obviously correct
definition against which the HIP path is checked. Only `tests/`,
`__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py` may import it.
It shares no code with the GPU library, and the GPU library never calls it.

The paper (Novotny, Adamek and Armour, "Implementing CUDA Streams into
AstroAccelerate - A Case Study") names the two phases it streams: dedispersion
(section 2.1) and the single-pulse search SPDT (section 2.2). It states no
formulas. The definitions below follow the method the paper's pipeline
implements: brute-force incoherent dedispersion (a shift-and-add over channels)
and a boxcar S/N search. Where the paper is silent, the readings listed in each
module header apply. All arithmetic is int64, exact Python integers or float64,
with the rounding points written out.

Modules:
  plan      channel frequencies, the float64 shift table, output sizes
  dedisp    D[d][t] = sum_c X[c][t + s[d][c]]
  sps       per-block moments, boxcar sums, S/N, best width, 3x3 peaks, candidates
  pipeline  whole-signal run and chunked run (section 1's time chunking)
  decimate  per-range time decimation: halvings of the input, range plans, their run
  cluster   cross-DM friends-of-friends clustering of a candidate list
"""

from .plan import K_DM, channel_freqs, shift_table, sizes
from .dedisp import dedisperse, dedisperse_rows
from .sps import block_moments, block_norms, best_plane, boxcar_strides, candidates, clipped_moments, single_pulse
from .pipeline import run, run_chunked
from .decimate import decimate, decimate2, range_plans, run_ranges
from .cluster import cluster

__all__ = ["K_DM", "channel_freqs", "shift_table", "sizes", "dedisperse", "dedisperse_rows",
           "block_moments", "block_norms", "best_plane", "boxcar_strides", "candidates", "clipped_moments", "single_pulse",
           "run", "run_chunked", "decimate", "decimate2", "range_plans", "run_ranges", "cluster"]
