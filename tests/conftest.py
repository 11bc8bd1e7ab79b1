import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large inputs (full-size workloads)")
    config.addinivalue_line("markers", "sanitize: host code and the oracle built with ASan/UBSan (CPU only)")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O

    O.lib()
    return O
