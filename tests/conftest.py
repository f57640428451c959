import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The oracle runs its cell loops on OpenMP threads. Under pytest-xdist every
# worker would start one thread per core; share the cores out instead (set
# before any test module loads the oracle library).
_workers = os.environ.get("PYTEST_XDIST_WORKER_COUNT")
if _workers and "OMP_NUM_THREADS" not in os.environ:
    os.environ["OMP_NUM_THREADS"] = str(max(1, (os.cpu_count() or 1) // int(_workers)))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
