import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


import pytest  # noqa: E402


@pytest.fixture(scope="session")
def csc():
    """The HIP library's Python binding; fails loudly when the library or the GPU is missing."""
    import torch

    import paper_1706_03591_amd as pkg

    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible MI355X")
    return pkg
