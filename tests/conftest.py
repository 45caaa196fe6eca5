import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_parts():
    """Build the oracle and the input evaluator if nothing is built yet."""
    import oracle
    from bto_inputs import _turb

    if not os.path.exists(oracle._LIB):
        oracle.build()
    if not os.path.exists(_turb._LIB):
        _turb.build()
    yield
