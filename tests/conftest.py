import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    # the oracle's C sweep is test infrastructure: build it once per session
    from oracle.build import build
    if not os.path.exists(os.path.join(ROOT, "oracle", "_oracle_sweep.so")):
        build()
    yield
