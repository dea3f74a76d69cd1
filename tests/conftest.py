import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library's C ABI)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def rebk():
    """The HIP library binding; on a GPU run a missing library is an error, never a skip."""
    import torch
    import paper_2001_04179_amd as rebk
    from paper_2001_04179_amd import _native
    _native.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return rebk
