import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _one_oracle_thread_per_xdist_worker():
    """Under pytest-xdist every worker runs the oracle at once: one OpenMP
    thread each (a test that wants more sets them and restores one), since
    oversubscribed thread teams stall at every parallel loop's barrier."""
    if os.environ.get("PYTEST_XDIST_WORKER"):
        import oracle
        oracle.set_threads(1)
    yield
