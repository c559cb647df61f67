import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running oracle check")


@pytest.fixture(scope="session")
def lib():
    from paper_2208_10907_amd import h2ulv
    return h2ulv.lib()
