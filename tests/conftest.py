import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X); parity tests of the HIP path")
    config.addinivalue_line("markers", "slow: full-size workload")


@pytest.fixture(scope="session")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _device_error_bits(request):
    """After every GPU test: no kernel may have raised a device-side error bit
    (read from the library's host word without a synchronisation, after the
    device has been synchronised here)."""
    yield
    if request.node.get_closest_marker("gpu") is None:
        return
    import torch
    if not torch.cuda.is_available():
        return
    import paper_2005_12648_amd as im
    torch.cuda.synchronize()
    im.device_status()
