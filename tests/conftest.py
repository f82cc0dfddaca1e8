import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def npg():
    from paper_2010_01775_amd import npg as _npg
    _npg.load_library()
    return _npg


@pytest.fixture(scope="session")
def ctx(npg):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    c = npg.Context(0)
    yield c
    c.close()
