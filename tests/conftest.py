import gc
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import build, oracle
    build.build()
    oracle._lib = None
    oracle._load()
    return oracle


@pytest.fixture(autouse=True)
def _collect_garbage_between_tests():
    """Destroy unreferenced library objects (plans and contexts, whose destructors free device
    memory) between tests, instead of whenever the cyclic collector next runs, which could be
    inside a later test's HIP-graph capture."""
    yield
    gc.collect()
