import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than ~20 s on the CPU")


@pytest.fixture(scope="session")
def gpu_ctx():
    """One LGF context on cuda:0 shared by the GPU tests."""
    import torch
    from paper_2010_13213_amd import lgf
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.init()
    ctx = lgf.Context(0)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()
