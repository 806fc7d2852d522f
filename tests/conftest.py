import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def dtlib():
    """The HIP library through its Python binding; a GPU test fails loudly
    if the library is not built."""
    # torch first: its HIP runtime is the one the library then binds to
    # (the tests hand it device tensors too)
    import torch
    if torch.cuda.is_available():
        torch.cuda.init()
    from paper_1902_07554_amd import binding
    binding.load()
    return binding
