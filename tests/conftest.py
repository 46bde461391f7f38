import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def rsr_ctx():
    """One library context on cuda:0 for the whole GPU session.  Fails (does not
    skip) when no GPU is visible: GPU tests must run the HIP path."""
    import torch
    import paper_2604_17066_amd as R
    assert torch.cuda.is_available(), "GPU test run without a visible HIP device"
    ctx = R.Context(0)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()
