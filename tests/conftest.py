import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    # progress lines of long steps (the full-size oracle runs) go to the real
    # stdout even while pytest captures the test's output
    from tests import _util
    _util.CAPTURE = config.pluginmanager.getplugin("capturemanager")


@pytest.fixture(scope="session")
def gpu_lib():
    """The loaded HIP library; GPU tests fail loudly when it is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2002_08014_amd import _lib
    return _lib.load()
