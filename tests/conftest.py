import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (gfx950) and the built libgabor")


@pytest.fixture(scope="session")
def gpu_lib():
    """The GPU binding; fails loudly (never falls back) when the library or
    the device is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu test selected but no GPU is visible")
    from paper_1704_05231_amd import binding
    binding.load()
    return binding
