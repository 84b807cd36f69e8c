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
    """Print what names each GPU case before it runs (a crash then still names it)."""
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(pytest.mark.usefixtures("_announce_gpu_case"))


@pytest.fixture
def _announce_gpu_case(request):
    sys.stdout.write(f"\n[gpu case] {request.node.nodeid}\n")
    sys.stdout.flush()
    yield
