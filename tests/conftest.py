import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~10 s")


@pytest.fixture(scope="session")
def lib():
    """The HIP library binding.  Tests load what is built and build only if
    nothing is."""
    from paper_2501_05110_amd import vfp
    if not os.path.exists(vfp.LIB_PATH):
        from paper_2501_05110_amd import build
        build.build(verbose=False)
    return vfp.load()


@pytest.fixture(scope="session")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")
