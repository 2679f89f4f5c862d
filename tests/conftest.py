import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


@pytest.fixture(scope="session")
def gpu_ctx():
    """One libkrt context on cuda:0 for the whole GPU session (fails loudly if the
    library is missing: there is no CPU fallback)."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2608_09340_amd import krt
    ctx = krt.Context(0)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()
