"""Seeded synthetic inputs: uint8 filterbanks with dispersed pulses, and DM-trial lists.

This package is shared test and benchmark infrastructure. Both the CPU oracle
tests and the GPU path draw their inputs from it. It holds none of the
dedispersion or single-pulse-search arithmetic: no shift table, no channel sums,
no boxcars, no S/N. The only physics it contains is the signal model, i.e. the
cold-plasma dispersion law that places a pulse in each channel at its continuous
(unrounded) arrival time. That law describes the sky, not the search method.
"""

from .dmplan import dm_plan
from .filterbank import Pulse, make_filterbank, random_pulses
from .workloads import WORKLOADS, workload

__all__ = ["dm_plan", "Pulse", "make_filterbank", "random_pulses", "WORKLOADS", "workload"]
