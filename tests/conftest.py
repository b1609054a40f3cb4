import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line(
        "markers", "slow: CPU test taking more than a few seconds")


def pytest_collection_modifyitems(config, items):
    # GPU tests run in file order; nothing to reorder here, the hook only
    # keeps the marker registration in one place.
    return None


@pytest.fixture(scope="session")
def repo_root():
    return ROOT


@pytest.fixture(scope="session", autouse=True)
def _torch_sees_the_gpu_first(request):
    """GPU tests that hand torch tensors to the library need torch's HIP
    runtime to initialise the device before the library's own runtime does
    (the other order leaves torch without devices).  Session scope runs this
    before any module fixture creates a library context."""
    if any(it.get_closest_marker("gpu") is not None for it in request.session.items):
        import torch
        if torch.cuda.is_available():
            torch.zeros(1, device="cuda")
    yield
