import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libpc2.so")
    config.addinivalue_line("markers", "slow: long-running oracle checks")


@pytest.fixture(scope="session")
def gpu_ctx():
    """One libpc2 context for the whole GPU session (skips when no GPU)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_14980_amd import pc2
    ctx = pc2.Context(0)
    yield ctx
    ctx.close()
