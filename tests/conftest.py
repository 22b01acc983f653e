import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# the batched form's tuner keeps its choices in a file: tests use one of
# their own, so that they neither read nor change the user's
if "PTMI_TUNE_CACHE" not in os.environ:
    import tempfile
    os.environ["PTMI_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="ptmi-tests-"), "tuning.txt")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle
