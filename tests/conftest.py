import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Compile the oracle once if it is not built yet (it is test infrastructure)."""
    from oracle.oracle import _LIB, build_oracle
    if not os.path.exists(_LIB):
        build_oracle()
    yield
