"""Runs GPU tests against the host-only sanitizer build of the library.

Usage (with the sanitizer runtime preloaded, as ``test_hostcheck_cpu.py``
does):  python tests/hostcheck/run_suite.py [pytest args ...]

``torch`` is replaced by ``fake_torch`` and the binding loads
``_build/hostcheck/libpchase_hostcheck.so``.  Kernels do not run, so the
tests' value checks fail; what this run checks is that the library's host
code, called in the tests' order, makes no invalid memory access, no
undefined behaviour and no misuse of the HIP runtime.  The skip marks of the
selected tests are lifted.  The process exits with pytest's status (0 or 1
when the run completed) and with a signal or the sanitizers' status when the
host code failed.
"""
from __future__ import annotations

import ctypes
import faulthandler
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from tests.hostcheck import build as hc_build  # noqa: E402
from tests.hostcheck import fake_torch  # noqa: E402


class LiftSkips:
    def pytest_collection_modifyitems(self, items):
        for item in items:
            for node in item.listchain():
                node.own_markers[:] = [m for m in node.own_markers if m.name != "skip"]


def main(argv):
    faulthandler.enable()
    lib = ctypes.CDLL(hc_build.LIB)
    fake_torch.bind(lib)
    sys.modules["torch"] = fake_torch
    from paper_1509_02308_amd import capi
    capi.LIB_PATH = hc_build.LIB
    capi._lib = None
    import pytest
    rc = pytest.main(["-p", "no:cacheprovider", "-q", "-m", "gpu", "--timeout", "600", "--timeout-method", "signal",
                      *argv], plugins=[LiftSkips()])
    capi.lib().pchase_release()
    left = lib.hostcheck_device_bytes()
    lib.hostcheck_calls.restype = ctypes.c_long
    lib.hostcheck_sites.restype = ctypes.c_long
    print(f"hostcheck: pytest status {int(rc)}, fallible runtime calls {lib.hostcheck_calls()} "
          f"from {lib.hostcheck_sites()} call sites, "
          f"device bytes still allocated after pchase_release: {left}", flush=True)
    return int(rc)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
