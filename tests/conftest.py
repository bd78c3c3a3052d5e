import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running statistical or full-size test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def tnmc():
    """The HIP library binding; with a GPU present a missing library is an error."""
    if not gpu_available():
        pytest.skip("no GPU visible")
    import paper_2509_19006_amd as lib
    lib.load()
    return lib
