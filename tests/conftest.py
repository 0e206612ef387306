import os
import sys

# The oracle's dense matrices in the tests are small (at most a few thousand
# rows): one BLAS thread per process is faster than a pool whose threads spin
# against each other and against other processes (a 256x256 test took 150 s
# with the default pool on a busy host, 2 s with one thread).  The variables
# cover libraries loaded later; threadpool_limits those already loaded.
for _var in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_var] = "1"

import numpy  # noqa: E402
import pytest  # noqa: E402
import scipy.linalg  # noqa: E402,F401
from threadpoolctl import threadpool_limits  # noqa: E402

_BLAS_LIMIT = threadpool_limits(limits=1, user_api="blas")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
