import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library bound through its C ABI (skips without a GPU)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_00308_amd as ps
    ps.load()   # raises if the native library is missing
    return ps
