import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test taking more than ~20 s")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP-backed binding; GPU tests fail loudly (not skip) when it cannot load."""
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    from paper_2112_10059_amd import binding
    binding.load()
    return binding
