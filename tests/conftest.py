import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def gpu_lib():
    """The loaded HIP library on a machine with a GPU (skips otherwise)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_00790_amd as bm
    bm.load()
    return bm
