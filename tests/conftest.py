import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def lne():
    """The GPU library binding; fails loudly when the native library is absent."""
    import paper_2302_07084_amd as lne_mod
    lne_mod.load()
    return lne_mod


@pytest.fixture(scope="session")
def ctx(lne):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lne.Context()


def to_dev(g):
    import torch
    return (torch.from_numpy(g.rowptr.astype("int64")).cuda(),
            torch.from_numpy(g.col.astype("int32")).cuda())
