import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct MI355X (gfx950) GPU")
    # the reference CPU transport is plain C; build it when it is missing
    lib = os.path.join(ROOT, "oracle", "liboracle.so")
    if not os.path.exists(lib):
        from oracle import build as obuild
        obuild.build()


@pytest.fixture(scope="session")
def root():
    return ROOT


@pytest.fixture(scope="session")
def gctx():
    """One libgdpm context on GPU 0 for the whole GPU test session."""
    from paper_1107_3355_amd import gdpm as G
    from paper_1107_3355_amd import inputs as I
    ctx = G.Context(0, materials=I.MATERIALS)
    yield ctx
    ctx.close()
