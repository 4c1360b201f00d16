import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long CPU test")
    # The CPU-only selection runs the oracle on small grids, whose steps are
    # thousands of short OpenMP regions: one thread unless the caller chose a
    # count (on a shared host, one descheduled thread would stall every
    # region's barrier).  Read by the OpenMP runtime when the oracle's
    # library is first loaded, which happens inside the tests.
    if "not gpu" in (config.getoption("markexpr", "") or "").replace("  ", " "):
        os.environ.setdefault("OMP_NUM_THREADS", "1")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import fimref
    return fimref.lib()
