import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running oracle check")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def ttr():
    """The HIP library binding; GPU tests fail loudly if it cannot load."""
    if not gpu_available():
        pytest.skip("no GPU visible")
    from paper_2011_06532_amd import ttr as lib
    lib.load()  # raises if libttr.so is missing
    return lib
