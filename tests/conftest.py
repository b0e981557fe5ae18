import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU run")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import build
    lib = build.LIB
    src = build.SRC
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        build.build()
    yield
