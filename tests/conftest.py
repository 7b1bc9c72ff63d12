import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X")
    config.addinivalue_line("markers", "slow: oracle runs of tens of seconds")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import forward
    if not os.path.exists(forward.LIB_PATH):
        from oracle.build import build
        build()
    yield
