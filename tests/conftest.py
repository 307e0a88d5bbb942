import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    """The loaded GPU library; a GPU test fails loudly if the HIP library or
    the device is missing instead of falling back to anything else."""
    if not _gpu_available():
        pytest.fail("gpu test run without a visible GPU")
    import paper_1804_11174_amd as kde
    kde.require_library()
    return kde
