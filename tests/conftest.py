import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: oracle work above a few seconds")


@pytest.fixture(scope="session")
def systems():
    """Cache of oracle systems per configuration name."""
    from oracle.operators import System
    from synthetic import get_config

    cache = {}

    def get(name, **overrides):
        key = (name, tuple(sorted((k, repr(v)) for k, v in overrides.items())))
        if key not in cache:
            cache[key] = System(get_config(name, **overrides))
        return cache[key]

    return get


def _ensure_built():
    here = os.path.join(ROOT, "paper_2202_11945_amd", "lib", "libfewha.so")
    if not os.path.exists(here):
        from __graft_entry__ import build
        build()


@pytest.fixture(scope="session")
def lib():
    """The built library (built once if missing)."""
    _ensure_built()
    import paper_2202_11945_amd as pkg
    return pkg


@pytest.fixture(scope="session")
def gpu_lib(lib):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a HIP device")
    return lib
