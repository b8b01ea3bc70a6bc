import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device); parity tests of the HIP path")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_built():
    from oracle import build
    if not (os.path.exists(os.path.join(ROOT, "oracle", "liborc.so"))
            and os.path.exists(os.path.join(ROOT, "oracle", "liborc_cs.so"))):
        build.build()
    return True


@pytest.fixture
def progress(capsys):
    """Print a line past pytest's output capture, at once: long GPU tests report each finished
    stage (a run of a thousand steps, say), so that a run under -q shows where it is."""
    def say(*args):
        with capsys.disabled():
            print(*args, flush=True)
    return say
