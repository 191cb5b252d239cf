import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    """The HIP binding; GPU tests fail loudly if the library is missing."""
    if not _gpu_available():
        pytest.skip("no GPU visible")
    from paper_1711_10855_amd import fdas
    fdas.load()  # raises if the shared library is absent
    return fdas
