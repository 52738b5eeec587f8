import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


_CACHE = {}


def workload(name, **kw):
    """Generated workloads are cached per process (generation is seeded)."""
    import lrgen
    key = (name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = lrgen.cached(name, **kw)
    return _CACHE[key]
