import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built GPU library; fails (does not skip) when it is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2607_22484_amd as psvt
    psvt.load()
    return psvt
