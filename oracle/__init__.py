"""CPU oracle of the P-chase cache-model replay (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (plain C,
single-threaded) through ctypes and shares no code with the HIP library.

Functions follow the paper (Mei & Chu, "Dissecting GPU Memory Hierarchy
through Microbenchmarking"):

* :func:`trace` -- Listing 1 + Listing 2: j <- A[j] with A[i] = (i+s) mod N.
* :func:`trace_nu` -- Section 5.2 / Fig. 13(b): the non-uniform-stride chase.
* :func:`replay` -- Section 4.1 set-associative model (Assumptions 1-3),
  plus the non-LRU policies of Sections 4.5/4.6.
* :func:`replay_general` -- the organisations of Sections 4.3-4.5 that break
  those assumptions: per-set associativity (L2 TLB), a set table (texture
  L1), weighted random replacement (Fermi L1).
* :func:`classify`, :func:`auto_threshold` -- Section 4.1, t = t0 + tm*r.
* :func:`infer` -- Section 4.2 / Fig. 6, as an exhaustive exact search.
* :func:`philox` -- Philox4x32-10 (Salmon et al., SC'11).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LRU, FIFO, PLRU, RANDOM, WRANDOM = 0, 1, 2, 3, 4


class OrcModel(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("capacity", "line", "ways", "sets", "policy", "set_shift", "seed")]


class OrcNuProbe(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("n_bytes", "base", "j0", "elem", "passes", "n_segments")]


class OrcGeneral(ctypes.Structure):
    _fields_ = [("line", ctypes.c_uint64), ("sets", ctypes.c_uint64), ("ways", ctypes.c_void_p),
                ("policy", ctypes.c_uint64), ("set_shift", ctypes.c_uint64), ("table_len", ctypes.c_uint64),
                ("table", ctypes.c_void_p), ("weights", ctypes.c_void_p), ("seed", ctypes.c_uint64)]


class OrcProbe(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("n_bytes", "s_bytes", "base", "j0", "elem", "passes")]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u64, i64, p = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [p, p, p]
        L.orc_trace_len.argtypes = [ctypes.POINTER(OrcProbe)]
        L.orc_trace_len.restype = u64
        L.orc_cycle_len.argtypes = [ctypes.POINTER(OrcProbe)]
        L.orc_cycle_len.restype = u64
        L.orc_trace.argtypes = [ctypes.POINTER(OrcProbe), p, u64]
        L.orc_trace.restype = u64
        L.orc_trace_nu_len.argtypes = [ctypes.POINTER(OrcNuProbe), p]
        L.orc_trace_nu_len.restype = u64
        L.orc_trace_nu.argtypes = [ctypes.POINTER(OrcNuProbe), p, p, p, u64]
        L.orc_trace_nu.restype = u64
        L.orc_general_check.argtypes = [ctypes.POINTER(OrcGeneral)]
        L.orc_general_check.restype = ctypes.c_int
        L.orc_replay_general.argtypes = [ctypes.POINTER(OrcGeneral), p, u64, u64, u64, u64, u64, p, p, p]
        L.orc_replay_general.restype = ctypes.c_int
        L.orc_model_check.argtypes = [ctypes.POINTER(OrcModel)]
        L.orc_model_check.restype = ctypes.c_int
        L.orc_replay.argtypes = [ctypes.POINTER(OrcModel), p, u64, u64, u64, u64, u64, p, p, p]
        L.orc_replay.restype = ctypes.c_int
        L.orc_classify.argtypes = [p, u64, ctypes.c_uint32, p]
        L.orc_auto_threshold.argtypes = [p, u64]
        L.orc_auto_threshold.restype = ctypes.c_uint32
        L.orc_infer.argtypes = [p, u64, p, u64, p, p, p, ctypes.c_int, p, p]
        L.orc_infer.restype = i64
        L.orc_infer_general.argtypes = [p, u64, p, u64, p, p, p, p, p]
        L.orc_infer_general.restype = i64
        L.orc_in_own_sweep.argtypes = [ctypes.POINTER(OrcModel), ctypes.POINTER(OrcProbe)]
        L.orc_in_own_sweep.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_model(C, b, a, policy=LRU, T=None, set_shift=0, seed=0) -> OrcModel:
    """Model tuple; T defaults to C/(a*b) (Assumption 1)."""
    if T is None:
        T = C // (a * b) if a * b and C % (a * b) == 0 else 0
    return OrcModel(C, b, a, T, policy, set_shift, seed)


def make_probe(N, s, passes=2, j0=0, base=0, elem=4) -> OrcProbe:
    return OrcProbe(N, s, base, j0, elem, passes)


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def cycle_len(probe: OrcProbe) -> int:
    return int(lib().orc_cycle_len(ctypes.byref(probe)))


def trace_len(probe: OrcProbe) -> int:
    return int(lib().orc_trace_len(ctypes.byref(probe)))


def trace(probe: OrcProbe) -> np.ndarray:
    n = trace_len(probe)
    if n == 0:
        raise ValueError("invalid probe")
    out = np.empty(n, dtype=np.int32)
    got = lib().orc_trace(ctypes.byref(probe), _ptr(out), n)
    assert got == n
    return out


def trace_nu(N, segments, passes=1, j0=0, base=0, elem=4) -> np.ndarray:
    """Section 5.2 non-uniform-stride chase; segments = [(s_bytes, count), ...]."""
    s = np.ascontiguousarray([int(x[0]) for x in segments], dtype=np.uint64)
    c = np.ascontiguousarray([int(x[1]) for x in segments], dtype=np.uint64)
    pr = OrcNuProbe(N, base, j0, elem, passes, len(segments))
    n = int(lib().orc_trace_nu_len(ctypes.byref(pr), _ptr(c))) if len(segments) else 0
    if n == 0:
        raise ValueError("invalid non-uniform probe")
    out = np.empty(n, dtype=np.int32)
    got = lib().orc_trace_nu(ctypes.byref(pr), _ptr(s), _ptr(c), _ptr(out), n)
    if got != n:
        raise ValueError("invalid non-uniform probe")
    return out


class General:
    """A generalised cache (see oracle.h): line bytes, per-set ways, policy,
    optional set_shift, set table and WRANDOM weights.  Keeps its arrays
    alive for the C struct."""

    def __init__(self, line, ways, policy=LRU, set_shift=0, table=None, weights=None, seed=0):
        self.ways = np.ascontiguousarray(ways, dtype=np.uint64)
        self.table = None if table is None else np.ascontiguousarray(table, dtype=np.uint64)
        self.weights = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint64)
        self.line, self.policy, self.set_shift, self.seed = int(line), int(policy), int(set_shift), int(seed)
        self.c = OrcGeneral(self.line, len(self.ways), _ptr(self.ways), self.policy, self.set_shift,
                            0 if self.table is None else len(self.table),
                            None if self.table is None else _ptr(self.table),
                            None if self.weights is None else _ptr(self.weights), self.seed)

    def ok(self) -> bool:
        return lib().orc_general_check(ctypes.byref(self.c)) == 0


def replay_general(g: General, idx, base=0, elem=4, trace_id=0, count_from=0):
    """Returns (hits uint8[len], misses_total, misses_steady)."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    hits = np.empty(max(len(idx), 1), dtype=np.uint8)
    mt = ctypes.c_uint64()
    ms = ctypes.c_uint64()
    rc = lib().orc_replay_general(ctypes.byref(g.c), _ptr(idx), len(idx), base, elem, trace_id,
                                  count_from, _ptr(hits), ctypes.byref(mt), ctypes.byref(ms))
    if rc != 0:
        raise ValueError(f"orc_replay_general failed ({rc})")
    return hits[: len(idx)], int(mt.value), int(ms.value)


def model_ok(model: OrcModel) -> bool:
    return lib().orc_model_check(ctypes.byref(model)) == 0


def replay(model: OrcModel, idx, base=0, elem=4, trace_id=0, count_from=0):
    """Returns (hits uint8[len], misses_total, misses_steady)."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    hits = np.empty(max(len(idx), 1), dtype=np.uint8)
    mt = ctypes.c_uint64()
    ms = ctypes.c_uint64()
    rc = lib().orc_replay(ctypes.byref(model), _ptr(idx), len(idx), base, elem, trace_id,
                          count_from, _ptr(hits), ctypes.byref(mt), ctypes.byref(ms))
    if rc != 0:
        raise ValueError(f"orc_replay failed ({rc})")
    return hits[: len(idx)], int(mt.value), int(ms.value)


def classify(lat, theta: int) -> np.ndarray:
    lat = np.ascontiguousarray(lat, dtype=np.uint32)
    out = np.empty(max(len(lat), 1), dtype=np.uint8)
    lib().orc_classify(_ptr(lat), len(lat), theta, _ptr(out))
    return out[: len(lat)]


def auto_threshold(lat) -> int:
    lat = np.ascontiguousarray(lat, dtype=np.uint32)
    return int(lib().orc_auto_threshold(_ptr(lat), len(lat)))


def in_own_sweep(model: OrcModel, probe: OrcProbe) -> bool:
    return bool(lib().orc_in_own_sweep(ctypes.byref(model), ctypes.byref(probe)))


def infer(cands, probes, obs_hits, obs_off, count_from, probe_select=1):
    """Exhaustive inference.  Returns (best or -1, m uint64[n], n uint64[n])."""
    nc, npb = len(cands), len(probes)
    carr = (OrcModel * max(nc, 1))(*cands)
    parr = (OrcProbe * max(npb, 1))(*probes)
    obs_hits = np.ascontiguousarray(obs_hits, dtype=np.uint8)
    obs_off = np.ascontiguousarray(obs_off, dtype=np.uint64)
    count_from = np.ascontiguousarray(count_from, dtype=np.uint64)
    m = np.zeros(max(nc, 1), dtype=np.uint64)
    n = np.zeros(max(nc, 1), dtype=np.uint64)
    best = lib().orc_infer(ctypes.cast(carr, ctypes.c_void_p), nc, ctypes.cast(parr, ctypes.c_void_p),
                           npb, _ptr(obs_hits), _ptr(obs_off), _ptr(count_from), probe_select,
                           _ptr(m), _ptr(n))
    if best < -1:
        raise ValueError(f"orc_infer failed ({best})")
    return int(best), m[:nc], n[:nc]


def infer_general(cands, probes, obs_hits, obs_off, count_from):
    """Exhaustive inference over General candidates, every probe for every
    candidate.  Returns (best or -1, m uint64[n], n uint64[n])."""
    nc, npb = len(cands), len(probes)
    carr = (OrcGeneral * max(nc, 1))(*[g.c for g in cands])
    parr = (OrcProbe * max(npb, 1))(*probes)
    obs_hits = np.ascontiguousarray(obs_hits, dtype=np.uint8)
    obs_off = np.ascontiguousarray(obs_off, dtype=np.uint64)
    count_from = np.ascontiguousarray(count_from, dtype=np.uint64)
    m = np.zeros(max(nc, 1), dtype=np.uint64)
    n = np.zeros(max(nc, 1), dtype=np.uint64)
    best = lib().orc_infer_general(ctypes.cast(carr, ctypes.c_void_p), nc, ctypes.cast(parr, ctypes.c_void_p),
                                   npb, _ptr(obs_hits), _ptr(obs_off), _ptr(count_from), _ptr(m), _ptr(n))
    if best < -1:
        raise ValueError(f"orc_infer_general failed ({best})")
    return int(best), m[:nc], n[:nc]


def zero_class(m) -> np.ndarray:
    """Indices of candidates reproducing the observation exactly."""
    return np.nonzero(np.asarray(m) == 0)[0]
