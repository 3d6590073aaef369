import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library through its C ABI)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


# The oracle's small tensor contractions are slower with a multi-threaded BLAS.
try:
    from threadpoolctl import threadpool_limits

    threadpool_limits(limits=1)
except ImportError:  # pragma: no cover
    pass
