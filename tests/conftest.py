import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU statistics")


@pytest.fixture(scope="session")
def gpu():
    """Skip unless a GPU is present; the HIP library must then load (no fallback)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_14688_amd as spin
    spin.load_library()
    return spin
