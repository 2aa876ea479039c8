import ctypes
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Keep freed heap memory for reuse: large numpy temporaries otherwise go
# back to the OS and every new one pays first-touch page faults again.
try:
    _libc = ctypes.CDLL("libc.so.6")
    _libc.mallopt(-1, 2 ** 31 - 1)   # M_TRIM_THRESHOLD
    _libc.mallopt(-2, 1 << 28)       # M_TOP_PAD
except OSError:
    pass


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle
    if not os.path.exists(oracle._LIB):
        oracle.build()
    return oracle
