import os
import sys
from functools import lru_cache

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI)")
    config.addinivalue_line("markers", "slow: CPU test taking more than ~10 s")


@lru_cache(maxsize=None)
def cube(n, seed=1, jitter=0.2):
    import synth
    return synth.jittered_cube(n, seed, jitter)


@lru_cache(maxsize=None)
def cube_geometry(n, seed=1, jitter=0.2):
    from oracle.geometry import build_geometry
    m = cube(n, seed, jitter)
    return build_geometry(m.xyz, m.tets, m.btris, m.btags)
