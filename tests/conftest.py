import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# The oracle's matrices are small: one BLAS thread runs them fastest, and a
# full-width thread pool per test process only adds overhead.
# The libraries are loaded first: the limit applies to those loaded.
try:
    import numpy  # noqa: F401
    import scipy.linalg  # noqa: F401
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1, user_api="blas")
except ImportError:
    pass
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")
