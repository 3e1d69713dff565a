import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle.lib()


@pytest.fixture(params=["fused", "general"])
def path(request):
    """GPU tests taking this fixture run twice: with the library's defaults (small
    images take the one-workgroup path) and with the general kernels only."""
    if request.param == "general":
        from tests.gpu_util import general_path
        with general_path():
            yield request.param
    else:
        yield request.param
