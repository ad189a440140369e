import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built libgs.so")
    config.addinivalue_line("markers", "slow: long CPU-oracle runs (minutes)")


@pytest.fixture(scope="session")
def gpu_ctx():
    """Library context on device 0. On a GPU machine a missing library or
    device is an error, never a skip."""
    import torch
    from paper_2602_17950_amd import gs
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    ctx = gs.Context(0)
    yield ctx
    ctx.close()
