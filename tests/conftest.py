import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU and the built libcitron.so")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def citron_gpu():
    """The product package, with a GPU present (GPU tests only)."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2112_10913_amd as citron
    citron.load_library()
    return citron


@pytest.fixture
def progress(request):
    """print() that bypasses output capture, so that a long GPU test shows
    its progress while it runs."""
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(*a):
        if capman is None:
            print(*a, flush=True)
            return
        with capman.global_and_fixture_disabled():
            print(*a, flush=True)
    return say
