import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def lsp():
    """The HIP library binding; GPU tests fail loudly if it cannot be loaded."""
    if not gpu_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    import paper_2102_08514_amd as pkg
    return pkg
