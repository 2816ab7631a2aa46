import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

# Under pytest-xdist every worker would otherwise start the oracle's OpenMP
# threads and the BLAS threads on all cores; spinning threads of several
# workers then starve each other and the suite crawls.  Each worker gets its
# share of the cores (settings made by the caller are kept).
if os.environ.get("PYTEST_XDIST_WORKER"):
    _workers = max(1, int(os.environ.get("PYTEST_XDIST_WORKER_COUNT", "1")))
    _share = str(max(1, (os.cpu_count() or 1) // _workers))
    for _var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ.setdefault(_var, _share)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU statistics runs")
