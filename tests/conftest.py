import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the host")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP solver bound through its C ABI; fails loudly if the library is missing."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("gpu test collected without a GPU")
    from paper_2008_08825_amd import api

    api.load_library()
    return api
