import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu on the GPU box)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def native():
    """The HIP library on a GPU; a GPU test never falls back to anything else."""
    import torch

    from paper_2402_02273_amd import _native

    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    return _native.lib()
