"""Writes the stored expected values in this folder. It calls only `oracle` (and the
seeded `synth` inputs). Run from the repository root: python tests/golden/make_golden.py"""

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth.workloads import make_input, workload  # noqa: E402


def main():
    w = workload("tiny_128ch_32k")
    x = make_input(w)
    r = oracle.run(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"],
                   w["threshold"], w["stat_block"])
    with open(os.path.join(HERE, "tiny_candidates.txt"), "w") as f:
        f.write("# tiny_128ch_32k: oracle candidates (dm_idx t width snr_f32), written by make_golden.py\n")
        f.write(f"# maxshift {r['sizes']['maxshift']} n_dd {r['sizes']['n_dd']} n_start {r['sizes']['n_start']}\n")
        for d, t, wd, snr in r["candidates"]:
            f.write(f"{d} {t} {wd} {snr!r}\n")


if __name__ == "__main__":
    main()
