import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built liblbm.so")
    config.addinivalue_line("markers", "slow: long-running oracle pin (still part of the CPU suite)")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on a real device; GPU tests fail loudly if either is missing."""
    import torch
    import paper_1410_2569_amd as L
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    L.lib()
    return L
