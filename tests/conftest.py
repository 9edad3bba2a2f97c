import os
import sys

import pytest

_BLAS_LIMIT = None

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")
    # The CPU suite's oracle runs work on small matrices, where BLAS thread
    # pools cost far more than they save (a CFET4 convergence test takes 20 s
    # on eight threads and 1.6 s on one; pytest-xdist workers would multiply
    # the pools further).  GPU runs keep the pools for their large references.
    global _BLAS_LIMIT
    if "not gpu" in (config.getoption("markexpr", "") or ""):
        import numpy  # noqa: F401  (load the BLAS libraries before limiting their pools)
        import scipy.linalg  # noqa: F401
        try:
            from threadpoolctl import threadpool_limits
        except ImportError:  # pragma: no cover
            return
        _BLAS_LIMIT = threadpool_limits(1)


def pytest_collection_modifyitems(config, items):
    # Keep GPU tests out of a CPU-only run unless explicitly asked for.
    pass
