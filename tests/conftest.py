import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X) and the built liblk.so")


@pytest.fixture(scope="session")
def ctx():
    """Library context on cuda:0 (GPU tests only)."""
    import paper_2106_12655_amd as lk
    return lk.Context(0)
