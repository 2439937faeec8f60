import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu():
    """The ctypes binding of the HIP library, on a machine with a GPU."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_10262_amd as lib
    lib.load()   # raises if the HIP library is not built: never a silent fallback
    return lib
