import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.fixture(scope="session")
def oracle_native():
    from oracle import native
    native.build(force=False)
    return native


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Name each GPU case on stdout (flushed) before it touches the device."""
    if request.node.get_closest_marker("gpu") is not None:
        print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    yield


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def mc():
    """The HIP library binding; fails (not skips) if the library is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_13679_amd as mcl
    from paper_2005_13679_amd import _lib
    _lib.load()
    return mcl
