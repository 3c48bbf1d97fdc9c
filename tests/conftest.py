import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def pytest_sessionstart(session):
    # The oracle multiplies many small blocks: multithreaded BLAS only adds contention
    # (and oversubscribes the host when several test processes run), so one thread each.
    try:
        from threadpoolctl import threadpool_limits
        session.config._blas_limits = threadpool_limits(limits=1)
    except ImportError:
        pass
