import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")


@pytest.fixture(scope="session")
def tiny():
    from synth.workloads import make_input, workload
    w = workload("tiny_128ch_32k")
    return w, make_input(w)


@pytest.fixture(scope="session")
def tiny_oracle(tiny):
    import oracle
    w, x = tiny
    return oracle.run(x, w["nsamp"], w["f_top"], w["foff"], w["tsamp"], w["dms"], w["widths"],
                      w["threshold"], w["stat_block"], want_best=True)
