import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def ico():
    """Cached icosphere meshes and oracle RWG tables by level."""
    from paper_2606_13482_amd.inputs import icosphere
    from oracle.mesh import rwg_table
    cache = {}

    def get(level):
        if level not in cache:
            V, T = icosphere(level)
            cache[level] = rwg_table(V, T)
        return cache[level]
    return get


@pytest.fixture(scope="session")
def bie():
    """The library binding; GPU tests skip without a device."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_13482_amd import bie as b
    return b
