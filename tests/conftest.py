import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Name every GPU case on the real stderr before it touches the device, so a
    run that ends abruptly still shows which case was running."""
    if request.node.get_closest_marker("gpu"):
        line = f"[gpu-case] start {request.node.nodeid}\n"
        path = os.environ.get("SCOCG_TEST_PROGRESS")
        if path:
            with open(path, "a") as f:
                f.write(line)
        sys.__stderr__.write(line)
        sys.__stderr__.flush()
    yield
