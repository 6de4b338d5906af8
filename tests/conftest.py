import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running statistical check")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.lib()
    return oracle


@pytest.fixture
def progress(capsys):
    """Prints a progress line past pytest's output capture, so that a long
    test still writes to the terminal while it runs under -q."""

    def say(*a):
        with capsys.disabled():
            print(*a, flush=True)

    return say
