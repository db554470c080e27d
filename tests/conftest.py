import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library on the device)")
    config.addinivalue_line("markers", "slow: long CPU oracle run (still part of the default suite)")


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle


@pytest.hookimpl(hookwrapper=True)
def pytest_runtest_makereport(item, call):
    """A device error (LBM_EDEVICE: the HIP runtime reported a fault) ends the session at
    once, so no further test touches a faulted GPU; ordinary failures let the run continue."""
    outcome = yield
    if call.excinfo is not None:
        exc = call.excinfo.value
        if type(exc).__name__ == "LbmError" and getattr(exc, "status", None) == -4:
            pytest.exit("device error in %s: %s" % (item.nodeid, exc), returncode=3)
