import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (runs the HIP library through the C ABI)")
    config.addinivalue_line(
        "markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def tiny0():
    from ofm_inputs import tiny_chain
    return tiny_chain(0)


@pytest.fixture(scope="session")
def tiny0_oracle(tiny0):
    import oracle as O
    s = tiny0
    return O.run(s.potential(), s.grid.h, s.frag_lo, s.frag_dims,
                 s.frag_states)
