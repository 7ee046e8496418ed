import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def library_built():
    """Build libatsparse.so (host cross-compile) if the tree has none at all;
    an existing build is used as is (rebuilding after a source change is the
    job of the build step, not of the tests)."""
    from paper_2012_08141_amd import build as lb
    if not os.path.exists(lb.LIB):
        lb.build()
    return True


@pytest.fixture(scope="session")
def oracle_built():
    from oracle import build as ob
    if not ob.built():
        ob.build()
    return True
