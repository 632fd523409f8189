import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


_MESHES = {}
_OPS = {}


@pytest.fixture(scope="session")
def oracle_mesh():
    import oracle

    def get(level):
        if level not in _MESHES:
            _MESHES[level] = oracle.Mesh(level)
        return _MESHES[level]
    return get


@pytest.fixture(scope="session")
def oracle_ops(oracle_mesh):
    import oracle

    def get(level, **kw):
        key = (level, tuple(sorted(kw.items())))
        if key not in _OPS:
            _OPS[key] = oracle.Ops(oracle_mesh(level), **kw)
        return _OPS[key]
    return get
