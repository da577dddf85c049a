import os
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import build as ob
    src = ob.SRC
    lib = ob.LIB
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        ob.build()
    yield
