import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: large-size case (full benchmark shapes)")


@pytest.fixture(scope="session")
def ss():
    """The HIP library binding; GPU tests only."""
    import paper_2004_12532_amd as m
    return m
