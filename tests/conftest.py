import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build(force=True)
    yield
    # the measures the GPU tests recorded, written as JSON to the file that
    # DFRSW_METRICS names (if set)
    from tests import gpu_util
    path = os.environ.get("DFRSW_METRICS")
    if gpu_util.METRICS and path:
        gpu_util.dump_metrics(path)
