"""C-ABI checks that need no GPU: every symbol declared in include/pchase.h
is exported by the built library, and malformed arguments are rejected on
the host (before anything would touch a device) with the documented codes."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pchase.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted({n for n in names if not n.startswith("sizeof")})


@pytest.fixture(scope="module")
def capi():
    from paper_1509_02308_amd import capi as C
    if not os.path.exists(C.LIB_PATH):
        pytest.fail("libpchase.so is not built (run __graft_entry__.build())")
    C.lib()
    return C


def test_header_functions_exported(capi):
    names = _declared_functions()
    assert {"pchase_trace", "cache_replay_batch", "infer_cache_params", "microbench_pchase",
            "microbench_hbm_stream", "microbench_lds_bank"} <= set(names)
    L = capi.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layouts_match_header(capi):
    assert ctypes.sizeof(capi.PchaseModel) == 40
    assert ctypes.sizeof(capi.PchaseProbe) == 40
    assert ctypes.sizeof(capi.PchaseResult) == 56
    assert ctypes.sizeof(capi.PchaseSegment) == 16
    assert ctypes.sizeof(capi.PchaseNuProbe) == 40
    assert ctypes.sizeof(capi.PchaseGeneralModel) == 56
    assert ctypes.sizeof(capi.PchasePlanChoice) == 24


def _rc(capi, rc):
    return rc, capi.last_error()


def test_trace_len_validation(capi):
    L = capi.lib()
    n, c = ctypes.c_uint64(), ctypes.c_uint64()
    ok = capi.PchaseProbe(52, 4, 0, 0, 4, 6)        # Fig. 3 array, 13 words
    assert L.pchase_trace_len(ctypes.byref(ok), ctypes.byref(n), ctypes.byref(c)) == 0
    assert (n.value, c.value) == (78, 13)
    for bad in (capi.PchaseProbe(10, 4, 0, 0, 4, 1),        # N not a multiple of elem
                capi.PchaseProbe(16, 6, 0, 0, 4, 1),        # s not a multiple of elem
                capi.PchaseProbe(16, 4, 0, 4, 4, 1),        # j0 outside
                capi.PchaseProbe(16, 4, 0, 0, 4, 0),        # no passes
                capi.PchaseProbe(16, 4, 0, 0, 8, 1),        # elem != 4
                capi.PchaseProbe(16, 4, 2, 0, 4, 1),        # misaligned base
                capi.PchaseProbe(1 << 33, 4, 0, 0, 4, 1)):  # N/elem >= 2^31
        rc = L.pchase_trace_len(ctypes.byref(bad), None, None)
        assert rc == -1, capi.last_error()
        assert capi.last_error()


@pytest.mark.parametrize("row,code", [
    ((4096, 32, 4, 4, 0, 0, 0), -1),      # unknown policy
    ((4096, 32, 3, 0, 0, 0, 0), -1),      # T*a*b != C
    ((4096, 24, 4, 0, 0, 0, 0), -1),      # line not a power of two
    ((6144, 32, 6, 2, 0, 0, 0), -1),      # PLRU with 6 ways
    ((4096, 32, 4, 0, 3, 0, 0), -1),      # set unit smaller than a line
    ((4096, 32, 4, 0, 0, 1, 0), -1),      # reserved field
    ((8192 * 32, 32, 256, 0, 0, 0, 0), -2),  # ways above 128
])
def test_model_validation_before_launch(capi, row, code):
    C, b, a, pol, sh, res, seed = row
    T = C // (a * b) if C % (a * b) == 0 else 1
    m = (capi.PchaseModel * 1)(capi.PchaseModel(C, b, a, T, pol, sh, res, seed))
    p = capi.probes([(4096, 32, 2)])
    pm = (ctypes.c_uint32 * 1)(0)
    pp = (ctypes.c_uint32 * 1)(0)
    rc = capi.lib().cache_replay_probes(ctypes.cast(m, ctypes.c_void_p), 1, ctypes.cast(p, ctypes.c_void_p), 1,
                                        pm, pp, None, 1, ctypes.c_void_p(16), None, None, 0, None, None)
    assert rc == code, capi.last_error()


def test_pair_index_validation(capi):
    m = capi.models([(4096, 32, 4, 0)])
    p = capi.probes([(4096, 32, 2)])
    pm = (ctypes.c_uint32 * 1)(1)                       # model index out of range
    pp = (ctypes.c_uint32 * 1)(0)
    rc = capi.lib().cache_replay_probes(ctypes.cast(m, ctypes.c_void_p), 1, ctypes.cast(p, ctypes.c_void_p), 1,
                                        pm, pp, None, 1, ctypes.c_void_p(16), None, None, 0, None, None)
    assert rc == -1 and "out of range" in capi.last_error()
    rc = capi.lib().cache_replay_probes(ctypes.cast(m, ctypes.c_void_p), 1, ctypes.cast(p, ctypes.c_void_p), 1,
                                        pp, pp, None, 1, ctypes.c_void_p(16), ctypes.c_void_p(16), None, 0, None, None)
    assert rc == -1 and "bitoff" in capi.last_error()
    rc = capi.lib().cache_replay_probes(ctypes.cast(m, ctypes.c_void_p), 1, ctypes.cast(p, ctypes.c_void_p), 1,
                                        pp, pp, None, 1, ctypes.c_void_p(16), None, None, 7, None, None)
    assert rc == -1 and "mode" in capi.last_error()


def test_trace_capacity_checked(capi):
    p = capi.probes([(4096, 4, 2)])                      # 2048 accesses
    off = (ctypes.c_uint64 * 2)()
    rc = capi.lib().pchase_trace(ctypes.cast(p, ctypes.c_void_p), 1, ctypes.c_void_p(16), off, 100, None)
    assert rc == -2 and "capacity" in capi.last_error()


def test_infer_argument_checks(capi):
    cands = capi.models([(4096, 32, 4, 0)])
    probes = capi.probes([(4096, 32, 2)])
    obs = capi.PchaseObservation(ctypes.cast(probes, ctypes.c_void_p), 1, capi.U32_MAX, None, None, None,
                                 None, None)
    res = capi.PchaseResult()
    L = capi.lib()
    # neither bits nor latencies
    rc = L.infer_cache_params(ctypes.byref(obs), ctypes.cast(cands, ctypes.c_void_p), 1, 1, 0, 8, None,
                              ctypes.byref(res), None, None, None, None)
    assert rc == -1 and "exactly one" in capi.last_error()
    # learned without a network
    rc = L.infer_cache_params(ctypes.byref(obs), ctypes.cast(cands, ctypes.c_void_p), 1, 1, 1, 8, None,
                              ctypes.byref(res), None, None, None, None)
    assert rc == -1
    rc = L.infer_cache_params(ctypes.byref(obs), ctypes.cast(cands, ctypes.c_void_p), 0, 1, 0, 8, None,
                              ctypes.byref(res), None, None, None, None)
    assert rc == -1 and "candidates" in capi.last_error()


def test_microbench_argument_checks(capi):
    L = capi.lib()
    assert L.microbench_lds_bank(0, 4, 1, ctypes.c_void_p(16), None) == -1
    assert L.microbench_lds_bank(4, 65, 1, ctypes.c_void_p(16), None) == -1
    g = ctypes.c_double()
    assert L.microbench_hbm_stream(ctypes.c_void_p(16), ctypes.c_void_p(16), 100, 1, 1, 64, 1, 1,
                                   ctypes.byref(g), None) == -1          # not a multiple of 16
    assert L.microbench_hbm_stream(ctypes.c_void_p(16), ctypes.c_void_p(16), 128, 0, 1, 64, 3, 1,
                                   ctypes.byref(g), None) == -1          # ilp 3
    p = capi.PchaseProbe(4096, 4, 0, 0, 4, 1)
    ovh = ctypes.c_int32()
    assert L.microbench_pchase(ctypes.byref(p), 0, ctypes.c_void_p(16), 1024, 10, ctypes.c_void_p(16),
                               ctypes.c_void_p(16), ctypes.byref(ovh), None) == -2   # array too small
    assert L.microbench_pchase(ctypes.byref(p), 9, ctypes.c_void_p(16), 8192, 10, ctypes.c_void_p(16),
                               ctypes.c_void_p(16), ctypes.byref(ovh), None) == -1   # flavour
    for args in ((0, 64, 1, 4, 0), (1, 100, 1, 4, 0), (1, 64, 3, 4, 0), (1, 64, 1, 8, 0), (1, 64, 1, 4, 2)):
        assert L.microbench_lds_stream(*args, 1, ctypes.byref(g), None) == -1
    assert L.microbench_valu(0, 1, ctypes.byref(g), None) == -1
    assert L.microbench_valu(1, 0, ctypes.byref(g), None) == -1


def test_nonuniform_trace_len_and_validation(capi, orc):
    """Host-only checks of the non-uniform chase (Section 5.2): the length
    agrees with the oracle; invalid probes are rejected before any launch."""
    rows = [(96, [(32, 1), (16, 1), (8, 1), (16, 1), (8, 2), (80, 1), (8, 3)], 3),
            (65 * (32 << 20), [(32 << 20, 260), (4, 64)], 2, 7)]
    parr, sarr = capi.nu_probes(rows)
    for i, r in enumerate(rows):
        n, K = capi.pchase_trace_nu_len(parr, sarr, i)
        assert n == len(orc.trace_nu(r[0], r[1], passes=r[2], j0=r[3] if len(r) > 3 else 0))
        assert K * r[2] == n
    L = capi.lib()
    n, K = ctypes.c_uint64(), ctypes.c_uint64()
    bad = [capi.nu_probes([(64, [(4, 0)])]),                 # empty segment
           capi.nu_probes([(64, [(6, 2)])]),                 # stride not a multiple of elem
           capi.nu_probes([(64, [(4, 2)], 1, 16)]),          # start outside the array
           capi.nu_probes([(64, [], 1)]),                    # no segment
           capi.nu_probes([(64, [(4, 1 << 31)], 2)])]        # 2^32 accesses
    for parr, sarr in bad:
        assert L.pchase_trace_nu_len(ctypes.byref(parr[0]), ctypes.cast(sarr, ctypes.c_void_p), sarr.n,
                                     ctypes.byref(n), ctypes.byref(K)) in (-1, -2)
    parr, sarr = capi.nu_probes([(64, [(4, 2)])])
    parr[0].first_segment = 1                                 # segment range outside the array
    assert L.pchase_trace_nu_len(ctypes.byref(parr[0]), ctypes.cast(sarr, ctypes.c_void_p), sarr.n,
                                 ctypes.byref(n), ctypes.byref(K)) == -1
    parr, sarr = capi.nu_probes([(4096, [(4, 1000)], 2)])
    off = (ctypes.c_uint64 * 2)()
    rc = L.pchase_trace_nu(ctypes.cast(parr, ctypes.c_void_p), 1, ctypes.cast(sarr, ctypes.c_void_p), 1,
                           ctypes.c_void_p(16), off, 100, None)
    assert rc == -2 and "capacity" in capi.last_error()


def test_general_model_validation_before_launch(capi):
    """Invalid generalised models are rejected on the host (no GPU needed)."""
    bad = [{"line": 48, "ways": [4]},                                  # line not a power of two
           {"line": 32, "ways": [4, 0]},                               # empty set
           {"line": 32, "ways": [200]},                                # more than 128 ways
           {"line": 32, "ways": [4, 3], "policy": 2},                  # PLRU needs 2^k ways
           {"line": 32, "ways": [4], "table": [0, 1]},                 # table entry outside the sets
           {"line": 32, "ways": [4], "policy": 4},                     # WRANDOM without weights
           {"line": 32, "ways": [2], "policy": 4, "weights": [0, 0]},  # zero total weight
           {"line": 32, "ways": [4], "policy": 5},                     # unknown policy
           {"line": 64, "ways": [4], "set_shift": 5}]                  # set unit below a line
    pm = (ctypes.c_uint32 * 1)(0)
    pt = (ctypes.c_uint32 * 1)(0)
    off = (ctypes.c_uint64 * 2)(0, 4)
    for d in bad:
        m = capi.general_models([d])
        rc = capi.lib().cache_replay_general(ctypes.cast(m, ctypes.c_void_p), 1, ctypes.c_void_p(16), off, None, 4,
                                             1, pm, pt, None, 1, ctypes.c_void_p(16), None, None, 0, None, None)
        assert rc == -1, d


def test_general_infer_argument_checks(capi):
    """The generalised search validates its candidates and observation on
    the host before it touches a device."""
    good = capi.general_models([{"line": 32, "ways": [4, 4]}])
    probes = capi.probes([(4096, 32, 2)])
    obs = capi.PchaseObservation(ctypes.cast(probes, ctypes.c_void_p), 1, capi.U32_MAX, None, None, None,
                                 None, None)
    res = capi.PchaseResult()
    L = capi.lib()
    rc = L.infer_cache_params_general(None, ctypes.cast(good, ctypes.c_void_p), 1, ctypes.byref(res), None, None,
                                      None, None)
    assert rc == -1
    rc = L.infer_cache_params_general(ctypes.byref(obs), ctypes.cast(good, ctypes.c_void_p), 0, ctypes.byref(res),
                                      None, None, None, None)
    assert rc == -1 and "candidates" in capi.last_error()
    rc = L.infer_cache_params_general(ctypes.byref(obs), ctypes.cast(good, ctypes.c_void_p), 1, ctypes.byref(res),
                                      None, None, None, None)
    assert rc == -1 and "exactly one" in capi.last_error()
    bad = capi.general_models([{"line": 32, "ways": [4, 3], "policy": 2}])
    rc = L.infer_cache_params_general(ctypes.byref(obs), ctypes.cast(bad, ctypes.c_void_p), 1, ctypes.byref(res),
                                      None, None, None, None)
    assert rc == -1 and "PLRU" in capi.last_error()


def test_planner_argument_checks(capi):
    """Planner arguments are checked on the host before any launch."""
    L = capi.lib()
    cands = capi.models([(4096, 32, 4, 0)])
    pool = capi.probes([(4096, 32, 2)])
    alive = (ctypes.c_uint32 * 1)(1)
    out = capi.PchasePlanChoice()
    vp = ctypes.c_void_p
    assert L.pchase_plan_next_probe(ctypes.cast(cands, vp), 0, ctypes.cast(pool, vp), 1, alive, None,
                                    ctypes.byref(out), None) == -1                       # no candidate
    assert L.pchase_plan_next_probe(ctypes.cast(cands, vp), 1, ctypes.cast(pool, vp), 0, alive, None,
                                    ctypes.byref(out), None) == -1                       # no probe
    assert L.pchase_plan_next_probe(ctypes.cast(cands, vp), 1, ctypes.cast(pool, vp), 1, None, None,
                                    ctypes.byref(out), None) == -1                       # no alive bitmap
    assert L.pchase_plan_next_probe(ctypes.cast(cands, vp), 9000, ctypes.cast(pool, vp), 1, alive, None,
                                    ctypes.byref(out), None) == -2                       # too many candidates
    bad = capi.models([(4096, 32, 3, 0)])                                                # T*a*b != C
    assert L.pchase_plan_next_probe(ctypes.cast(bad, vp), 1, ctypes.cast(pool, vp), 1, alive, None,
                                    ctypes.byref(out), None) == -1


def test_mlp_grid_matches_reference(capi):
    """The library's feature grid is the reference grid (host-only call)."""
    from oracle import mlp_ref
    arr = capi.pchase_mlp_grid(64)
    got = [(arr[i].n_bytes, arr[i].s_bytes, arr[i].passes) for i in range(768)]
    assert got == mlp_ref.grid()
    assert all(arr[i].base_offset == 64 and arr[i].j0 == 0 and arr[i].elem_bytes == 4 for i in range(768))
    with pytest.raises(capi.PchaseError):
        capi.pchase_mlp_grid(2)


def test_static_replay_argument_checks(capi):
    L = capi.lib()
    m = capi.models([(8192, 32, 4, 0)])
    off = np.array([0, 4], np.uint64)
    z = np.zeros(1, np.uint32)
    args = lambda eb: (ctypes.cast(m, ctypes.c_void_p), 1, None, off.ctypes.data, None, eb, 1, z.ctypes.data,
                       z.ctypes.data, None, 1, None, None, None, None)
    assert L.cache_replay_batch_static(*args(8)) == -1      # elem_bytes must be 4
    assert L.cache_replay_batch_static(*args(4)) == -1      # misses_dev is NULL
    bad = capi.models([(8192, 32, 3, 0)])                  # T*a*b != C
    assert L.cache_replay_batch_static(ctypes.cast(bad, ctypes.c_void_p), *args(4)[1:]) == -1


def test_plan_lifetime_without_device(capi):
    """Plans are created only on a usable device: here (no GPU) creation fails
    with ENODEV and leaves the handle NULL; a NULL out pointer or an empty
    reservation is EINVAL; destroying NULL is a no-op."""
    L = capi.lib()
    h = ctypes.c_void_p(1234)
    assert L.pchase_plan_create(1 << 20, ctypes.byref(h)) == -6
    assert not h.value
    assert L.pchase_plan_create(1 << 20, None) == -1
    assert L.pchase_plan_create(0, ctypes.byref(h)) == -1
    L.pchase_plan_destroy(None)
