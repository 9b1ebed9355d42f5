import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: full-size case, minutes of oracle time")


import pytest  # noqa: E402


@pytest.fixture(autouse=True)
def _clean_device_status(request):
    """After every GPU test: synchronise and require a clean device status
    word (no kernel of the test gave up a look-back wait)."""
    yield
    if request.node.get_closest_marker("gpu") is None:
        return
    import torch
    if not torch.cuda.is_available() or not torch.cuda.is_initialized():
        return
    from paper_2504_08624_amd import functional
    v = functional.device_status(clear=True)
    assert v == 0, "a kernel flagged a workspace during this test (status word 0x%x)" % v
