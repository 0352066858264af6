import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU run of the oracle")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    if not os.path.exists(O.LIB) or os.path.getmtime(O.LIB) < os.path.getmtime(O.SRC):
        O.build()
    return O


@pytest.fixture(scope="session")
def oracle3d_mod():
    from oracle import oracle3d as O3
    if not os.path.exists(O3.LIB) or os.path.getmtime(O3.LIB) < os.path.getmtime(O3.SRC):
        O3.build()
    return O3


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; the test is an error (not a
    silent skip) when the GPU or the library is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_1702_04487_amd import lbm
    lbm.load()
    return lbm
