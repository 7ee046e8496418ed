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
def private_caches(tmp_path_factory):
    """Caches the library and the compiler write (the autotuner's choices,
    compiled variants, the code-object compiler's own cache) go to a
    temporary directory for the session, not to the user's home."""
    d = str(tmp_path_factory.mktemp("cache"))
    old = {k: os.environ.get(k) for k in ("XDG_CACHE_HOME", "AMD_COMGR_CACHE_DIR")}
    os.environ["XDG_CACHE_HOME"] = d
    os.environ["AMD_COMGR_CACHE_DIR"] = os.path.join(d, "comgr")
    yield d
    for k, v in old.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


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
