import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on cuda:0; GPU tests need a visible MI355X."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1404_0027_amd import arsel

    arsel.context(0)
    return torch.device("cuda:0")
