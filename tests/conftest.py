import faulthandler
import os
import sys

import pytest

# a fault inside a native call prints the Python stack of every thread and,
# when the helper is built, the native stack first
faulthandler.enable()
_CRASH_TRACE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native", "libcrash_trace.so")
if os.path.exists(_CRASH_TRACE):
    import ctypes
    ctypes.CDLL(_CRASH_TRACE)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
