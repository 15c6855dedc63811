"""Host-only build of libpchase for the sanitizer checks of its host code.

Every ``csrc/*.hip`` file is compiled for the host side only (the kernels
become launch stubs), instrumented with AddressSanitizer and
UndefinedBehaviorSanitizer, and linked with ``hip_host_stub.cpp`` (a
stand-in for the HIP runtime) into ``_build/hostcheck/libpchase_hostcheck.so``.
Nothing here runs on, or is loaded by, the GPU build.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import re
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1509_02308_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(ROOT, "_build", "hostcheck")
LIB = os.path.join(OUT, "libpchase_hostcheck.so")
ROCM = "/opt/rocm"
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")

# the sanitizers apply to the host compilation only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
HOST_ONLY = ["-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def asan_runtime() -> str:
    hits = sorted(glob.glob(os.path.join(ROCM, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("clang's AddressSanitizer runtime is not installed")
    return hits[-1]


def symbolizer() -> str:
    return os.path.join(ROCM, "llvm", "bin", "llvm-symbolizer")


def available() -> bool:
    return os.path.exists(os.path.join(ROCM, "bin", "hipcc")) and os.path.exists(CLANG)


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{res.stderr}")
    return res


def _compile(src: str) -> str:
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    _run([os.path.join(ROCM, "bin", "hipcc"), *HOST_ONLY, *SAN, "-c", src, "-o", obj])
    return obj


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + [os.path.join(HERE, "hip_host_stub.cpp")]
    with concurrent.futures.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, srcs))
    # a host-only object refers to the device code object of its file by a
    # per-file symbol; the stand-in registers nothing from it, so an empty
    # definition of each suffices
    names = set()
    for o in objs:
        out = _run(["nm", "-u", o]).stdout
        names.update(re.findall(r"\b(__hip_fatbin_[0-9a-f]+)\b", out))
    fat = os.path.join(OUT, "fatbin_symbols.c")
    with open(fat, "w") as f:
        for n in sorted(names):
            f.write(f"const char {n}[8] = {{0}};\n")
    fat_o = fat + ".o"
    _run([CLANG, "-x", "c", "-fPIC", "-c", fat, "-o", fat_o])
    tmp = LIB + ".tmp"
    _run([CLANG, "-shared", "-fPIC", *SAN, "-shared-libsan", "-Wl,-Bsymbolic", "-o", tmp, *objs, fat_o,
          "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
