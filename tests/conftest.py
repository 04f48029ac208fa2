import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through libgbs.so)")


@pytest.fixture(scope="session")
def gpu_ctx():
    """A gbs context on cuda:0.  Fails loudly if the HIP library or GPU is missing."""
    import paper_2106_01445_amd as g
    g.load()
    ctx = g.Context(0)
    yield ctx
    ctx.close()
