import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU (MI355X)")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    return oracle.lib()


@pytest.fixture(scope="session")
def gomlib():
    """libgom.so, built only if it is missing."""
    from paper_2203_08680_amd import build as gbuild
    from paper_2203_08680_amd import gom
    if not os.path.exists(gom.LIB_PATH):
        gbuild.build()
    return gom.lib()


@pytest.fixture(scope="session")
def cuda(gomlib):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)
