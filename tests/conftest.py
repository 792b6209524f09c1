import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-only check")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built C-ABI library, on a machine with a GPU; skips elsewhere."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_06735_amd import _lib
    return _lib.load()
