import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


@pytest.fixture(scope="session")
def ora():
    """The CPU oracle (built on first use)."""
    from oracle import build as obuild
    from oracle import oracle as o
    if not os.path.exists(obuild.LIB):
        obuild.build()
    return o
