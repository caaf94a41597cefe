import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


import pytest  # noqa: E402


@pytest.fixture(scope="session")
def gpu_handle():
    """A librgs handle on cuda:0 bound to torch's current stream (GPU tests only)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_05090_amd as rgs
    h = rgs.Handle(0)
    yield h
    h.close()
