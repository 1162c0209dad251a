import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


_CACHE = {}


def workload(name, **kw):
    """Seeded synthetic workload, cached per session: (scene, probes, views)."""
    import synth
    key = (name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = synth.workload(name, **kw)
    return _CACHE[key]


@pytest.fixture(scope="session")
def tiny():
    return workload("tiny")


@pytest.fixture(scope="session")
def single_small():
    """The 8x8x4 / 128^2 room of the single-view workload, seen through a 240x135 view."""
    return workload("single", size=(240, 135))


def fp16_bits(a):
    return np.asarray(a, dtype=np.float16).view(np.uint16)
