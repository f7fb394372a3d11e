import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device); parity tests of the GPU path")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session", autouse=True)
def _cpu_libs():
    """The CPU-side test libraries (oracle, workload generator) are cheap g++ builds."""
    import oracle
    import workloads
    oracle.build()
    workloads.build()
    yield
