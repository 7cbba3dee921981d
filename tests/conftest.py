import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def gpu():
    """The HIP binding on cuda:0; the test fails if the GPU or the library is missing."""
    import torch
    from paper_2011_06787_amd import spiir
    if not torch.cuda.is_available():
        pytest.fail("gpu test selected but no GPU is visible")
    spiir.load()   # raises if the HIP library is missing
    return spiir
