import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running oracle comparison")


@pytest.fixture(scope="session")
def oracle_weights():
    """Kernel weights of the float64 oracle, shared by the full-size tests of one session
    (keyed as ``oracle.sbim.PlaneOperator`` keys them: q, c_s, dt, W, eta)."""
    return {}
