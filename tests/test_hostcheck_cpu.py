"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

``tests/hostcheck`` builds the library for the host only and links it with a
stand-in for the HIP runtime whose device memory is inaccessible to host
code, whose asynchronous copies run only when a synchronisation completes
them, and which records graph captures (its header lists what it checks).
The GPU tests are then run against that build, in their collection order,
with the sanitizer runtime preloaded: the kernels do not run, so their value
checks fail, and what must hold is that no sanitizer or stand-in check
fires.  A second pass makes one runtime call fail at each distinct call site
of a sequence of tests, so that the library's error returns run too.  The
first test plants mistakes in a small host program and checks that each is
caught, so that a clean run means something.
"""
from __future__ import annotations

import concurrent.futures
import os
import re
import subprocess
import sys
import textwrap

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
RUNNER = os.path.join(HERE, "hostcheck", "run_suite.py")

# every GPU test except the three whose oracle side takes minutes of CPU
FAST = ["tests/", "-k", "not full and not benchmark_size"]
# the order of a full GPU run that once ended in a host fault: edge cases,
# generalised caches, the large-batch shape, then the network's features
SEQUENCE = ["tests/test_gpu_edges.py", "tests/test_gpu_general.py",
            "tests/test_gpu_large_batch.py::test_large_batch_shape_matches_oracle",
            "tests/test_gpu_mlp.py::test_features_match_oracle"]


def _hb():
    from tests.hostcheck import build as hb
    return hb


@pytest.fixture(scope="module")
def lib():
    hb = _hb()
    if not hb.available():
        pytest.skip("hipcc or ROCm clang is not installed")
    return hb.build()


def _env(**extra):
    hb = _hb()
    env = dict(os.environ)
    env.update(LD_PRELOAD=hb.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=1:symbolize=1",
               ASAN_SYMBOLIZER_PATH=hb.symbolizer(),
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.update({k: str(v) for k, v in extra.items()})
    return env


def _run(args, timeout=900, **extra):
    return subprocess.run([sys.executable, RUNNER, "-s", *args], cwd=ROOT, env=_env(**extra), capture_output=True,
                          text=True, timeout=timeout)


def _findings(res):
    out = res.stdout + res.stderr
    bad = [ln for ln in out.splitlines()
           if ln.startswith("HOSTCHECK:") or "ERROR: AddressSanitizer" in ln or "runtime error:" in ln]
    if res.returncode not in (0, 1) or "hostcheck: pytest status" not in out:
        bad.append(f"exit status {res.returncode}; tail:\n" + "\n".join(out.splitlines()[-40:]))
    return bad


PLANTED = {
    # host code reads device memory
    "host_reads_device": ("""
        p = c_void_p(); L.hipMalloc(byref(p), 4096)
        string_at(p.value, 4)
        """, "SEGV"),
    # an asynchronous copy whose host source is freed before the stream completes
    "source_freed_before_sync": ("""
        p = c_void_p(); L.hipMalloc(byref(p), 1 << 20)
        a = np.ones(1 << 18, np.float32)
        L.hipMemcpyAsync(p, c_void_p(a.ctypes.data), c_size_t(1 << 20), 1, None)
        del a; gc.collect()
        L.hipStreamSynchronize(None)
        """, "heap-use-after-free"),
    # a copy into device memory freed earlier
    "copy_into_freed_device_memory": ("""
        p = c_void_p(); L.hipMalloc(byref(p), 4096); L.hipFree(p)
        a = np.ones(16, np.float32)
        L.hipMemcpy(p, c_void_p(a.ctypes.data), c_size_t(64), 1)
        """, "freed earlier"),
    # a copy past the end of a device allocation
    "copy_past_device_allocation": ("""
        p = c_void_p(); L.hipMalloc(byref(p), 100)
        a = np.ones(64, np.float32)
        L.hipMemcpy(p, c_void_p(a.ctypes.data), c_size_t(256), 1)
        """, "overruns"),
    # a copy kind that does not match the pointers
    "wrong_copy_kind": ("""
        p = c_void_p(); L.hipMalloc(byref(p), 4096)
        a = np.ones(16, np.float32)
        L.hipMemcpy(c_void_p(a.ctypes.data), p, c_size_t(64), 1)
        """, "HostToDevice copy"),
    # an allocation while a stream captures
    "allocation_during_capture": ("""
        s = c_void_p(); L.hipStreamCreateWithFlags(byref(s), 1)
        L.hipStreamBeginCapture(s, 2)
        p = c_void_p(); L.hipMalloc(byref(p), 4096)
        """, "while a stream captures"),
}


@pytest.mark.parametrize("case", sorted(PLANTED))
def test_stand_in_catches_planted_mistakes(lib, case):
    body, expect = PLANTED[case]
    prog = "import gc\nfrom ctypes import *\nimport numpy as np\n" \
           f"L = CDLL({lib!r})\n" + textwrap.dedent(body)
    res = subprocess.run([sys.executable, "-c", prog], env=_env(), capture_output=True, text=True, timeout=120)
    assert res.returncode != 0, (case, res.stdout, res.stderr)
    assert expect in res.stderr, (case, res.stderr[-3000:])


def test_gpu_suite_host_code_is_clean(lib):
    res = _run(FAST)
    assert not _findings(res), _findings(res)


def test_error_returns_of_the_sequence_are_clean(lib):
    """One failing runtime call per distinct call site of SEQUENCE."""
    res = _run(SEQUENCE)
    assert not _findings(res), _findings(res)
    n_sites = int(re.search(r"from (\d+) call sites", res.stdout).group(1))
    assert n_sites > 20

    def one(k):
        r = _run(SEQUENCE, timeout=300, HOSTCHECK_FAIL_SITE=k)
        return k, _findings(r)

    workers = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        bad = [(k, f) for k, f in ex.map(one, range(1, n_sites + 1)) if f]
    assert not bad, bad[:3]
