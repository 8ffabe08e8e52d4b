import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle check")

# The oracle works on small dense matrices (Krylov projections, 2^L <= 4096 blocks), where a
# multi-threaded BLAS spends far more time synchronising threads than computing: pin it to one.
try:
    from threadpoolctl import threadpool_limits

    _BLAS_LIMIT = threadpool_limits(limits=1)
except ImportError:  # pragma: no cover
    _BLAS_LIMIT = None
