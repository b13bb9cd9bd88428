import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; calls the HIP library through its C ABI")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_ctx():
    import torch
    from paper_1902_08018_amd import wh
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = wh.wh_create(0, 0)
    yield ctx
    wh.wh_destroy(ctx)
