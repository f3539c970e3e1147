import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: larger CPU oracle runs")


@pytest.fixture(scope="session")
def hip_device():
    """Skip unless a HIP device is visible; fail loudly if the library is missing."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2103_11962_amd import regmg

    regmg.load()  # raises if the shared library is not built
    return torch.device("cuda:0")
