import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


_CACHE = {}


def cached(key, fn):
    """Session-wide cache for expensive oracle objects."""
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]


@pytest.fixture(scope="session")
def sphere_oracle():
    from paper_2009_02281_amd import inputs as I
    from oracle.aimx import AimOracle

    def make():
        w = I.sphere_small()
        o = AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
        o.C  # assemble once
        return w, o
    return cached("sphere_small", make)
