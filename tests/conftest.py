import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle work of more than a few seconds")


def pytest_collection_finish(session):
    # The oracle's worker processes are forked here, after collection and
    # before any test runs, so that no worker inherits GPU state.
    if any("oracle_pool" in getattr(item, "fixturenames", ()) for item in session.items):
        from tests import oracle_pool
        oracle_pool.start()


def pytest_unconfigure(config):
    mod = sys.modules.get("tests.oracle_pool")
    if mod is not None:
        mod.stop()


@pytest.fixture(scope="session")
def oracle_pool():
    from tests import oracle_pool as P
    return P.get()
