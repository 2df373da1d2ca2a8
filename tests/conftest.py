import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built libpond.so")
    config.addinivalue_line("markers", "slow: long-running physics check")


@pytest.fixture(scope="session")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    # the product must load its own HIP library; no fallback
    from paper_1806_05089_amd import _lib
    _lib.load()
    return torch.device("cuda:0")
