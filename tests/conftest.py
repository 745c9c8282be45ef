import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Launch shapes the tests time (TVS_FLAG_AUTOTUNE) go to a file of the test session, not to the
# user's cache, unless the caller chose one.
if "TVS_TUNE_CACHE" not in os.environ:
    import tempfile

    os.environ["TVS_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="tvs-tests-"), "tune.txt")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running check (several seconds of oracle time)")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.lib()
    return oracle
