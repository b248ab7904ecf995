import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    return oracle


def small_workload(n=(7, 6, 5), length=(1.0, 0.8, 0.6), lo=(2, 2, 2), hi=(4, 3, 2),
                   material=None, loops=((1, 3, 1.0),), waveform=1, **kw):
    """A non-cubic box-conductor workload with square coil loops (d, k, I)."""
    import synth
    mat = material or synth.Material(1.0e6, 0.0, 0.0, synth.NU0)
    cm = synth.box_cell_mat(n, lo, hi)
    S = (n[0] + 1) * (n[1] + 1) * (n[2] + 1)
    xs = np.zeros(3 * S)
    for d, k, cur in loops:
        synth.square_loop(n, xs, d, k, cur)
    return synth.Workload(name="small", n=n, length=length, cell_mat=cm,
                          materials=[mat], edge_current=xs, waveform=waveform, **kw)
