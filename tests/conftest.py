import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU oracle physics run")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library on a machine with a GPU; builds it only if nothing is built."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_04443_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1908_04443_amd import build
        build.build()
    lbm.lib()
    return lbm
