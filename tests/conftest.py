import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    """Skip cleanly on a machine without a GPU; on a GPU machine, load the HIP
    library and fail loudly when it is missing."""
    if not _gpu_available():
        pytest.skip("no GPU on this machine")
    from paper_1404_0466_amd import binding
    binding.load()  # raises when the library is not built
    return binding
