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
    # Print the test id before each GPU test runs, so a crashed box still names its case.
    pass


@pytest.fixture(autouse=True)
def _announce_gpu_test(request):
    if request.node.get_closest_marker("gpu") is not None:
        sys.stdout.write(f"\n[gpu-test] {request.node.nodeid}\n")
        sys.stdout.flush()
    yield
