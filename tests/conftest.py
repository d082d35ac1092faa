import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests run in one process; nothing to reorder here beyond marking.
    pass


@pytest.fixture(scope="session")
def ctx():
    """A library context on cuda:0 (GPU tests only)."""
    import paper_2208_08410_amd as P
    c = P.Context(0)
    yield c
    c.close()
