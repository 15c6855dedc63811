"""Thin ctypes binding of libpchase (include/pchase.h), same names as the C ABI.

Argument marshalling only: every step of the replay, scoring and search runs
in the library's HIP kernels.  Device buffers are torch tensors on the
current device, streams are torch's current stream.  The binding raises if
the built library is missing; it never falls back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpchase.so")

PCHASE_OK = 0
LRU, FIFO, PLRU, RANDOM, WRANDOM = 0, 1, 2, 3, 4
BATCHED, PLAIN = 0, 1
PROBES_ALL, PROBES_OWN_SWEEP = 0, 1
EXHAUSTIVE, LEARNED = 0, 1
SCHED_PLAIN = 0x100
SCHED_UNTUNED = 0x200
SCHED_FULL_REPLAY = 0x400
LOAD_DEFAULT, LOAD_L2, LOAD_SYSTEM, LOAD_STREAM = 0, 1, 2, 3
MLP_IN, MLP_HIDDEN = 768, 256
U32_MAX = 0xFFFFFFFF

u32, u64, i32, i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
vp = ctypes.c_void_p


class PchaseModel(ctypes.Structure):
    _fields_ = [("capacity_bytes", u64), ("line_bytes", u32), ("ways", u32), ("sets", u32),
                ("policy", u32), ("set_shift", u32), ("reserved", u32), ("seed", u64)]


class PchaseProbe(ctypes.Structure):
    _fields_ = [("n_bytes", u64), ("s_bytes", u64), ("base_offset", u64), ("j0", u64),
                ("elem_bytes", u32), ("passes", u32)]


class PchaseGeneralModel(ctypes.Structure):
    _fields_ = [("line_bytes", u32), ("n_sets", u32), ("policy", u32), ("set_shift", u32),
                ("set_ways", vp), ("set_table", vp), ("table_len", u32), ("weights_len", u32),
                ("way_weights", vp), ("seed", u64)]


class PchasePlanChoice(ctypes.Structure):
    _fields_ = [("probe", i64), ("worst", u32), ("n_classes", u32), ("n_alive", u32), ("reserved", u32)]


class PchaseSegment(ctypes.Structure):
    _fields_ = [("s_bytes", u64), ("count", u64)]


class PchaseNuProbe(ctypes.Structure):
    _fields_ = [("n_bytes", u64), ("base_offset", u64), ("j0", u64), ("elem_bytes", u32), ("passes", u32),
                ("first_segment", u32), ("n_segments", u32)]


class PchaseObservation(ctypes.Structure):
    _fields_ = [("probes", vp), ("n_probes", u32), ("threshold", u32), ("bits_dev", vp),
                ("bitoff", vp), ("lat_dev", vp), ("lat_off", vp), ("count_from", vp)]


class PchaseResult(ctypes.Structure):
    _fields_ = [("best", i64), ("best_m", u64), ("best_n", u64), ("n_zero", u64),
                ("replayed_accesses", u64), ("closed_form_accesses", u64), ("fallback", u32),
                ("threshold_used", u32)]


class PchaseError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pchase error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run paper_1509_02308_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.pchase_last_error.restype = ctypes.c_char_p
        L.pchase_trace_len.argtypes = [ctypes.POINTER(PchaseProbe), vp, vp]
        L.pchase_trace.argtypes = [vp, u32, vp, vp, u64, vp]
        L.cache_replay_general.argtypes = [vp, u32, vp, vp, vp, u32, u32, vp, vp, vp, u64, vp, vp, vp, u32, vp, vp]
        L.pchase_plan_create.argtypes = [u64, ctypes.POINTER(vp)]
        L.pchase_plan_destroy.argtypes = [vp]
        L.pchase_plan_destroy.restype = None
        L.pchase_plan_next_probe.argtypes = [vp, u32, vp, u32, vp, vp, ctypes.POINTER(PchasePlanChoice), vp]
        L.pchase_trace_nu_len.argtypes = [ctypes.POINTER(PchaseNuProbe), vp, u32, vp, vp]
        L.pchase_trace_nu.argtypes = [vp, u32, vp, u32, vp, vp, u64, vp]
        L.cache_replay_batch.argtypes = [vp, u32, vp, vp, vp, u32, u32, vp, vp, vp, u64, vp, vp, vp, u32, vp, vp]
        L.cache_replay_batch_static.argtypes = [vp, u32, vp, vp, vp, u32, u32, vp, vp, vp, u64, vp, vp, vp, vp]
        L.cache_replay_probes.argtypes = [vp, u32, vp, u32, vp, vp, vp, u64, vp, vp, vp, u32, vp, vp]
        L.infer_cache_params.argtypes = [ctypes.POINTER(PchaseObservation), vp, u32, ctypes.c_int,
                                         ctypes.c_int, u32, vp, ctypes.POINTER(PchaseResult), vp, vp, vp, vp]
        L.infer_cache_params_general.argtypes = [ctypes.POINTER(PchaseObservation), vp, u32,
                                                 ctypes.POINTER(PchaseResult), vp, vp, vp, vp]
        L.microbench_pchase.argtypes = [ctypes.POINTER(PchaseProbe), u32, vp, u64, u64, vp, vp, vp, vp]
        L.pchase_microbench_max_k.restype = u64
        L.microbench_hbm_stream.argtypes = [vp, vp, u64, u32, u32, u32, u32, u32, vp, vp]
        L.microbench_lds_bank.argtypes = [u32, u32, u32, vp, vp]
        L.microbench_lds_stream.argtypes = [u32, u32, u32, u32, u32, u32, vp, vp]
        L.microbench_valu.argtypes = [u32, u32, vp, vp]
        L.pchase_abort.argtypes = [ctypes.c_int]
        L.pchase_release.argtypes = []
        L.pchase_mlp_grid.argtypes = [vp, u64]
        L.pchase_mlp_create.argtypes = [u32, u64, ctypes.POINTER(vp)]
        L.pchase_mlp_destroy.argtypes = [vp]
        L.pchase_mlp_destroy.restype = None
        L.pchase_mlp_features.argtypes = [vp, u32, vp, vp]
        L.pchase_mlp_labels.argtypes = [vp, u32, vp, vp]
        L.pchase_mlp_samples.argtypes = [vp, u32, vp, u64, u32, u64, u32, vp, vp, vp]
        L.pchase_mlp_train_step.argtypes = [vp, vp, vp, u32, ctypes.c_float, vp, vp]
        L.pchase_mlp_train.argtypes = [vp, vp, vp, u64, u32, u32, ctypes.c_float, vp, vp]
        L.pchase_mlp_forward.argtypes = [vp, vp, u32, vp, vp]
        L.pchase_mlp_topk.argtypes = [vp, u32, u32, u32, vp, vp]
        L.pchase_mlp_param.argtypes = [vp, u32, u32, vp, vp, ctypes.c_int]
        L.pchase_mlp_step_count.argtypes = [vp, vp, ctypes.c_int]
        _lib = L
    return _lib


def last_error() -> str:
    return lib().pchase_last_error().decode()


def check(rc: int):
    if rc != PCHASE_OK:
        raise PchaseError(rc, last_error())


# ------------------------------------------------------------- marshalling --
def _stream(stream=None):
    if stream is not None:
        return vp(stream)
    import torch
    return vp(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A caller-owned plan (pchase_plan_create / pchase_plan_destroy):
    device_bytes of workspace reserved once; the replay and inference calls
    given it allocate no device memory."""

    def __init__(self, device_bytes: int):
        h = vp()
        check(lib().pchase_plan_create(device_bytes, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().pchase_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _plan(plan):
    return plan.handle if plan is not None else None


def _dptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return vp(t.data_ptr())


def _hptr(a, dtype):
    """Host pointer of a numpy array kept alive by the caller (or None)."""
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr, arr.ctypes.data_as(vp)


def models(rows) -> ctypes.Array:
    """Model descriptors from (C, b, a, policy[, set_shift[, seed]]) rows or a
    workloads.MODEL_DT array; sets = C / (a*b) (Assumption 1)."""
    rows = list(rows)
    out = (PchaseModel * max(len(rows), 1))()
    for i, r in enumerate(rows):
        if isinstance(r, np.void):
            C, b, a, pol, sh, seed = (int(r["C"]), int(r["b"]), int(r["a"]), int(r["policy"]),
                                      int(r["set_shift"]), int(r["seed"]))
        else:
            r = tuple(int(x) for x in r) + (0,) * (6 - len(r))
            C, b, a, pol, sh, seed = r
        sets = C // (a * b) if a * b and C % (a * b) == 0 else 0
        out[i] = PchaseModel(C, b, a, sets, pol, sh, 0, seed)
    out.n = len(rows)
    return out


def probes(rows) -> ctypes.Array:
    """Probe descriptors from (N, s[, passes[, j0[, base]]]) rows or a
    workloads.PROBE_DT array (elem = 4 bytes)."""
    rows = list(rows)
    out = (PchaseProbe * max(len(rows), 1))()
    for i, r in enumerate(rows):
        if isinstance(r, np.void):
            N, s, base, j0, elem, passes = (int(r["N"]), int(r["s"]), int(r["base"]), int(r["j0"]),
                                            int(r["elem"]), int(r["passes"]))
        else:
            r = tuple(int(x) for x in r)
            N, s = r[0], r[1]
            passes = r[2] if len(r) > 2 else 2
            j0 = r[3] if len(r) > 3 else 0
            base = r[4] if len(r) > 4 else 0
            elem = 4
        out[i] = PchaseProbe(N, s, base, j0, elem, passes)
    out.n = len(rows)
    return out


def pchase_trace_len(probe: PchaseProbe):
    n, L = u64(), u64()
    check(lib().pchase_trace_len(ctypes.byref(probe), ctypes.byref(n), ctypes.byref(L)))
    return int(n.value), int(L.value)


def pchase_trace(probe_arr, idx, stream=None) -> np.ndarray:
    """Fills idx (int32 CUDA tensor) with the probes' traces; returns offsets."""
    off = np.zeros(probe_arr.n + 1, dtype=np.uint64)
    check(lib().pchase_trace(ctypes.cast(probe_arr, vp), probe_arr.n, _dptr(idx), off.ctypes.data_as(vp),
                             idx.numel() if idx is not None else 0, _stream(stream)))
    return off


def nu_probes(rows):
    """Non-uniform probe and segment arrays from rows
    (N, [(s_bytes, count), ...][, passes[, j0[, base]]]); each row gets its
    own run of segments.  Returns (probe array, segment array)."""
    rows = list(rows)
    segs = [sg for r in rows for sg in r[1]]
    parr = (PchaseNuProbe * max(len(rows), 1))()
    sarr = (PchaseSegment * max(len(segs), 1))()
    first = 0
    for i, r in enumerate(rows):
        N, sl = int(r[0]), r[1]
        passes = int(r[2]) if len(r) > 2 else 1
        j0 = int(r[3]) if len(r) > 3 else 0
        base = int(r[4]) if len(r) > 4 else 0
        parr[i] = PchaseNuProbe(N, base, j0, 4, passes, first, len(sl))
        for t, (s, c) in enumerate(sl):
            sarr[first + t] = PchaseSegment(int(s), int(c))
        first += len(sl)
    parr.n = len(rows)
    sarr.n = len(segs)
    return parr, sarr


def pchase_trace_nu_len(probe_arr, seg_arr, i=0):
    n, K = u64(), u64()
    check(lib().pchase_trace_nu_len(ctypes.byref(probe_arr[i]), ctypes.cast(seg_arr, vp), seg_arr.n,
                                    ctypes.byref(n), ctypes.byref(K)))
    return int(n.value), int(K.value)


def pchase_trace_nu(probe_arr, seg_arr, idx, stream=None) -> np.ndarray:
    """Fills idx (int32 CUDA tensor) with the non-uniform probes' traces;
    returns the offsets."""
    off = np.zeros(probe_arr.n + 1, dtype=np.uint64)
    check(lib().pchase_trace_nu(ctypes.cast(probe_arr, vp), probe_arr.n, ctypes.cast(seg_arr, vp), seg_arr.n,
                                _dptr(idx), off.ctypes.data_as(vp), idx.numel() if idx is not None else 0,
                                _stream(stream)))
    return off


def cache_replay_batch(model_arr, idx, trace_off, trace_base, pair_model, pair_trace, count_from,
                       misses, hitbits=None, bitoff=None, mode=BATCHED, stream=None, plan=None):
    toff, p_toff = _hptr(trace_off, np.uint64)
    tb, p_tb = _hptr(trace_base, np.uint64)
    pm, p_pm = _hptr(pair_model, np.uint32)
    pt, p_pt = _hptr(pair_trace, np.uint32)
    cf, p_cf = _hptr(count_from, np.uint64)
    bo, p_bo = _hptr(bitoff, np.uint64)
    check(lib().cache_replay_batch(ctypes.cast(model_arr, vp), model_arr.n, _dptr(idx), p_toff, p_tb, 4,
                                   len(toff) - 1, p_pm, p_pt, p_cf, len(pm), _dptr(misses), _dptr(hitbits),
                                   p_bo, mode, _plan(plan), _stream(stream)))


def cache_replay_batch_static(model_arr, idx, trace_off, trace_base, pair_model, pair_trace, count_from,
                              misses, hitbits=None, bitoff=None, stream=None):
    toff, p_toff = _hptr(trace_off, np.uint64)
    tb, p_tb = _hptr(trace_base, np.uint64)
    pm, p_pm = _hptr(pair_model, np.uint32)
    pt, p_pt = _hptr(pair_trace, np.uint32)
    cf, p_cf = _hptr(count_from, np.uint64)
    bo, p_bo = _hptr(bitoff, np.uint64)
    check(lib().cache_replay_batch_static(ctypes.cast(model_arr, vp), model_arr.n, _dptr(idx), p_toff, p_tb, 4,
                                          len(toff) - 1, p_pm, p_pt, p_cf, len(pm), _dptr(misses), _dptr(hitbits),
                                          p_bo, _stream(stream)))


def general_models(rows) -> ctypes.Array:
    """Generalised model descriptors from dicts with keys line, ways (list,
    one per set), policy, and optionally set_shift, table (list), weights
    (list) and seed.  The returned array keeps its host arrays alive."""
    rows = list(rows)
    out = (PchaseGeneralModel * max(len(rows), 1))()
    keep = []
    for i, r in enumerate(rows):
        ways = np.ascontiguousarray(r["ways"], dtype=np.uint32)
        table = None if r.get("table") is None else np.ascontiguousarray(r["table"], dtype=np.uint32)
        weights = None if r.get("weights") is None else np.ascontiguousarray(r["weights"], dtype=np.uint32)
        keep += [ways, table, weights]
        out[i] = PchaseGeneralModel(int(r["line"]), len(ways), int(r.get("policy", LRU)), int(r.get("set_shift", 0)),
                                    ways.ctypes.data, None if table is None else table.ctypes.data,
                                    0 if table is None else len(table), 0 if weights is None else len(weights),
                                    None if weights is None else weights.ctypes.data, int(r.get("seed", 0)))
    out.n = len(rows)
    out.keep = keep
    return out


def cache_replay_general(model_arr, idx, trace_off, trace_base, pair_model, pair_trace, count_from,
                         misses, hitbits=None, bitoff=None, mode=BATCHED, stream=None, plan=None):
    toff, p_toff = _hptr(trace_off, np.uint64)
    tb, p_tb = _hptr(trace_base, np.uint64)
    pm, p_pm = _hptr(pair_model, np.uint32)
    pt, p_pt = _hptr(pair_trace, np.uint32)
    cf, p_cf = _hptr(count_from, np.uint64)
    bo, p_bo = _hptr(bitoff, np.uint64)
    check(lib().cache_replay_general(ctypes.cast(model_arr, vp), model_arr.n, _dptr(idx), p_toff, p_tb, 4,
                                     len(toff) - 1, p_pm, p_pt, p_cf, len(pm), _dptr(misses), _dptr(hitbits),
                                     p_bo, mode, _plan(plan), _stream(stream)))


def cache_replay_probes(model_arr, probe_arr, pair_model, pair_probe, count_from, misses, hitbits=None,
                        bitoff=None, mode=BATCHED, stream=None, plan=None):
    pm, p_pm = _hptr(pair_model, np.uint32)
    pp, p_pp = _hptr(pair_probe, np.uint32)
    cf, p_cf = _hptr(count_from, np.uint64)
    bo, p_bo = _hptr(bitoff, np.uint64)
    check(lib().cache_replay_probes(ctypes.cast(model_arr, vp), model_arr.n, ctypes.cast(probe_arr, vp),
                                    probe_arr.n, p_pm, p_pp, p_cf, len(pm), _dptr(misses), _dptr(hitbits),
                                    p_bo, mode, _plan(plan), _stream(stream)))


def infer_cache_params(probe_arr, cand_arr, bits=None, bitoff=None, lat=None, lat_off=None,
                       threshold=U32_MAX, count_from=None, probe_select=PROBES_OWN_SWEEP,
                       mode=EXHAUSTIVE, topk=8, net=None, mn=None, want_zero=False, stream=None, plan=None):
    """Returns (PchaseResult, zero-class bitmap as uint32 array or None)."""
    bo, p_bo = _hptr(bitoff, np.uint64)
    lo, p_lo = _hptr(lat_off, np.uint64)
    cf, p_cf = _hptr(count_from, np.uint64)
    obs = PchaseObservation(ctypes.cast(probe_arr, vp), probe_arr.n, threshold, _dptr(bits), p_bo,
                            _dptr(lat), p_lo, p_cf)
    res = PchaseResult()
    zero = np.zeros((cand_arr.n + 31) // 32, dtype=np.uint32) if want_zero else None
    check(lib().infer_cache_params(ctypes.byref(obs), ctypes.cast(cand_arr, vp), cand_arr.n, probe_select,
                                   mode, topk, net.handle if net is not None else None, ctypes.byref(res), _dptr(mn),
                                   zero.ctypes.data_as(vp) if zero is not None else None,
                                   _plan(plan), _stream(stream)))
    return res, zero


def infer_cache_params_general(probe_arr, gen_arr, bits=None, bitoff=None, lat=None, lat_off=None,
                               threshold=U32_MAX, count_from=None, mn=None, want_zero=False, stream=None,
                               plan=None):
    """Generalised candidates (general_models(...)); returns (PchaseResult,
    zero-class bitmap as uint32 array or None)."""
    bo, p_bo = _hptr(bitoff, np.uint64)
    lo, p_lo = _hptr(lat_off, np.uint64)
    cf, p_cf = _hptr(count_from, np.uint64)
    obs = PchaseObservation(ctypes.cast(probe_arr, vp), probe_arr.n, threshold, _dptr(bits), p_bo,
                            _dptr(lat), p_lo, p_cf)
    res = PchaseResult()
    zero = np.zeros((gen_arr.n + 31) // 32, dtype=np.uint32) if want_zero else None
    check(lib().infer_cache_params_general(ctypes.byref(obs), ctypes.cast(gen_arr, vp), gen_arr.n,
                                           ctypes.byref(res), _dptr(mn),
                                           zero.ctypes.data_as(vp) if zero is not None else None,
                                           _plan(plan), _stream(stream)))
    return res, zero


def pchase_plan_next_probe(cand_arr, pool_arr, alive, classes=None, stream=None) -> PchasePlanChoice:
    """Next probe of the adaptive procedure for the surviving candidates
    (alive: uint32 bitmap words); classes (int32 CUDA tensor of
    n_pool * n_cands, optional) receives the class matrix."""
    a = np.ascontiguousarray(alive, dtype=np.uint32)
    out = PchasePlanChoice()
    check(lib().pchase_plan_next_probe(ctypes.cast(cand_arr, vp), cand_arr.n, ctypes.cast(pool_arr, vp), pool_arr.n,
                                       a.ctypes.data_as(vp), _dptr(classes), ctypes.byref(out), _stream(stream)))
    return out


def pchase_microbench_max_k() -> int:
    return int(lib().pchase_microbench_max_k())


def microbench_pchase(probe: PchaseProbe, flavor, array, k, lat, idx, stream=None) -> int:
    """idx None: no index records, 16-bit latencies (4x the capacity)."""
    ovh = i32()
    check(lib().microbench_pchase(ctypes.byref(probe), flavor, _dptr(array),
                                  array.numel() * array.element_size(), k, _dptr(lat), _dptr(idx),
                                  ctypes.byref(ovh), _stream(stream)))
    return int(ovh.value)


def microbench_hbm_stream(src, dst, nbytes, dtype, grid, block, ilp, reps, stream=None) -> float:
    g = ctypes.c_double()
    check(lib().microbench_hbm_stream(_dptr(src), _dptr(dst), nbytes, dtype, grid, block, ilp, reps,
                                      ctypes.byref(g), _stream(stream)))
    return float(g.value)


def microbench_lds_bank(stride_lo, stride_hi, reps, cycles, stream=None):
    check(lib().microbench_lds_bank(stride_lo, stride_hi, reps, _dptr(cycles), _stream(stream)))


def microbench_lds_stream(blocks_per_cu, block, ilp, width_bytes, reps, copy=False, stream=None) -> float:
    g = ctypes.c_double()
    check(lib().microbench_lds_stream(blocks_per_cu, block, ilp, width_bytes, int(bool(copy)), reps,
                                      ctypes.byref(g), _stream(stream)))
    return float(g.value)


def microbench_valu(blocks_per_cu=8, reps=20000, stream=None) -> float:
    """Measured 32-bit VALU lane operations per second."""
    g = ctypes.c_double()
    check(lib().microbench_valu(blocks_per_cu, reps, ctypes.byref(g), _stream(stream)))
    return float(g.value)


def pchase_abort(on: bool):
    lib().pchase_abort(1 if on else 0)


def pchase_release():
    check(lib().pchase_release())


# ------------------------------------------------------------ learned model --
def pchase_mlp_grid(base_offset=0) -> ctypes.Array:
    """The 768 feature-grid probes (host descriptors)."""
    arr = (PchaseProbe * MLP_IN)()
    check(lib().pchase_mlp_grid(ctypes.cast(arr, vp), base_offset))
    arr.n = MLP_IN
    return arr


def pchase_mlp_features(model_arr, x, stream=None):
    check(lib().pchase_mlp_features(ctypes.cast(model_arr, vp), model_arr.n, _dptr(x), _stream(stream)))


def pchase_mlp_labels(model_arr, stream=None) -> np.ndarray:
    out = np.zeros(model_arr.n, dtype=np.int32)
    check(lib().pchase_mlp_labels(ctypes.cast(model_arr, vp), model_arr.n, out.ctypes.data_as(vp),
                                  _stream(stream)))
    return out


def pchase_mlp_samples(model_arr, class_of_model, first, n, seed, rho_q16, x, labels, stream=None):
    cm, p_cm = _hptr(class_of_model, np.int32)
    check(lib().pchase_mlp_samples(ctypes.cast(model_arr, vp), model_arr.n, p_cm, first, n, seed, rho_q16,
                                   _dptr(x), _dptr(labels), _stream(stream)))


def pchase_mlp_topk(logits, k, idx, stream=None):
    rows, ncls = logits.shape
    check(lib().pchase_mlp_topk(_dptr(logits), rows, ncls, k, _dptr(idx), _stream(stream)))


class Mlp:
    """Owning handle of a pchase_mlp network (pchase_mlp_create/destroy)."""

    def __init__(self, n_out: int, seed: int):
        h = vp()
        check(lib().pchase_mlp_create(n_out, seed, ctypes.byref(h)))
        self.handle = h
        self.n_out = n_out

    def close(self):
        if self.handle:
            lib().pchase_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def train_step(self, x, labels, lr, want_loss=True, stream=None):
        loss = ctypes.c_float()
        check(lib().pchase_mlp_train_step(self.handle, _dptr(x), _dptr(labels), x.shape[0], lr,
                                          ctypes.byref(loss) if want_loss else None, _stream(stream)))
        return float(loss.value) if want_loss else None

    def train(self, x, labels, batch, epochs, lr, stream=None):
        loss = ctypes.c_float()
        check(lib().pchase_mlp_train(self.handle, _dptr(x), _dptr(labels), x.shape[0], batch, epochs, lr,
                                     ctypes.byref(loss), _stream(stream)))
        return float(loss.value)

    def forward(self, x, logits, stream=None):
        check(lib().pchase_mlp_forward(self.handle, _dptr(x), x.shape[0], _dptr(logits), _stream(stream)))

    def param(self, which, slot=0) -> np.ndarray:
        nb = u64()
        check(lib().pchase_mlp_param(self.handle, which, slot, None, ctypes.byref(nb), 0))
        out = np.zeros(nb.value // 4, dtype=np.float32)
        check(lib().pchase_mlp_param(self.handle, which, slot, out.ctypes.data_as(vp), ctypes.byref(nb), 0))
        return out

    def set_param(self, which, slot, values):
        arr = np.ascontiguousarray(values, dtype=np.float32).reshape(-1)
        nb = u64()
        check(lib().pchase_mlp_param(self.handle, which, slot, None, ctypes.byref(nb), 0))
        assert arr.nbytes == nb.value, (arr.nbytes, nb.value)
        check(lib().pchase_mlp_param(self.handle, which, slot, arr.ctypes.data_as(vp), ctypes.byref(nb), 1))

    def steps(self, value=None) -> int:
        v = u64(0 if value is None else value)
        check(lib().pchase_mlp_step_count(self.handle, ctypes.byref(v), 0 if value is None else 1))
        return int(v.value)
