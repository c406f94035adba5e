import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def skel():
    """The HIP library, initialised on cuda:0 with torch's caching allocator.
    Importing the package raises if libskel.so is missing (no fallback)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1405_2915_amd as sk
    sk.skel_init(0, "torch")
    import oracle
    oracle.set_threads(min(16, os.cpu_count() or 1))
    return sk
