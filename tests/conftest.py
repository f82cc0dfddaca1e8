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


@pytest.fixture(scope="session")
def clustered():
    """The clustered workload's 5e7 photons (generated once per session)."""
    from paper_2010_01775_amd import synth
    return synth.clustered_photons()


@pytest.fixture(scope="session")
def clustered_tree(orc, clustered):
    """The oracle's octree (split > 8192, depth <= 6) over those photons."""
    rc, ref = orc.build_tree(clustered.pos, 8192, 6, max_leaves=1 << 20)
    assert rc == 0
    return ref
