import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session", autouse=True)
def _oracle_c_kernel():
    """Build the oracle's small C kernel routine (gcc) if it is not there yet."""
    from oracle import kernel

    try:
        kernel.build()
    except Exception:  # the NumPy path of the same formula is used instead
        pass
    yield
