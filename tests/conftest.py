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
def _built_cpu_libs():
    """Build the oracle and the input generator if they are not built yet."""
    import oracle
    import seeded_inputs
    oracle.build(force=False)
    seeded_inputs.build(force=False)
    yield
