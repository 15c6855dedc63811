"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
own formula: they use the paper's worked examples, closed forms derived from
Assumptions 1-3, special cases, published Philox vectors, an independent
library (rocRAND) and brute force (oracle/brute.py) on tiny inputs.
"""
import os
import shutil
import subprocess
from fractions import Fraction
from math import gcd

import numpy as np
import pytest

from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))


# -------------------------------------------------------------- trace ----
@pytest.mark.parametrize("n,s,j0", [(13, 1, 0), (16, 4, 0), (12, 8, 3), (10, 15, 2),
                                    (7, 7, 0), (24, 9, 5), (5, 0, 1), (64, 96, 0)])
def test_trace_is_listing_1_and_2(orc, n, s, j0):
    """Listing 1 + Listing 2 run literally on an array give the same indices."""
    p = orc.make_probe(4 * n, 4 * s, passes=3, j0=j0)
    got = orc.trace(p).tolist()
    assert got == brute.listing_trace(n, s, len(got), j0)
    # one pass returns to the start: the sequence is periodic in the cycle length
    L = orc.cycle_len(p)
    assert got[L] == j0 and len(set(got[:L])) == L


def test_trace_rejects_bad_probes(orc):
    assert orc.trace_len(orc.make_probe(10, 4)) == 0       # N not a multiple of elem
    assert orc.trace_len(orc.make_probe(16, 6)) == 0       # s not a multiple of elem
    assert orc.trace_len(orc.make_probe(16, 4, j0=4)) == 0  # start outside the array
    assert orc.trace_len(orc.make_probe(16, 4, passes=0)) == 0


# ------------------------------------------ non-uniform stride (5.2) ----
def _fig13b():
    segs, visited, n = [], None, None
    with open(os.path.join(HERE, "golden", "fig13b_nonuniform_chase.txt")) as f:
        for line in f:
            w = line.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "n_elems":
                n = int(w[1])
            elif w[0] == "segment":
                segs.append((int(w[1]), int(w[2])))
            elif w[0] == "visited":
                visited = [int(x) for x in w[1:]]
    return n, segs, visited


def test_nonuniform_fig13b_example(orc):
    """Section 5.2, Fig. 13(b): the drawn array gives the drawn chase."""
    n, segs, visited = _fig13b()
    got = orc.trace_nu(4 * n, [(4 * st, c) for st, c in segs], passes=2)
    assert got.tolist() == visited * 2


@pytest.mark.parametrize("n,s,j0,passes", [(13, 1, 0, 3), (16, 4, 0, 2), (12, 8, 3, 2), (24, 9, 5, 3),
                                           (5, 0, 1, 2), (64, 96, 0, 2), (1000, 36, 17, 2)])
def test_nonuniform_one_segment_is_uniform(orc, n, s, j0, passes):
    """One segment of one full cycle is the Listing 1 + 2 chase."""
    L = n // gcd(n, s % n)
    got = orc.trace_nu(4 * n, [(4 * s, L)], passes=passes, j0=j0)
    assert got.tolist() == brute.listing_trace(n, s, passes * L, j0)


def test_nonuniform_matches_pointer_array(orc):
    """Random segment lists that an array can realise (each element at most
    once per pass): the chase over the explicitly initialised array."""
    rng = np.random.default_rng(5)
    done = 0
    for _ in range(400):
        n = int(rng.integers(8, 400))
        segs = [(int(rng.integers(0, 3 * n)), int(rng.integers(1, 6))) for _ in range(int(rng.integers(1, 6)))]
        j0 = int(rng.integers(0, n))
        K = sum(c for _, c in segs)
        want = brute.pointer_array_chase(n, segs, 3 * K, j0)
        if want is None:
            continue
        got = orc.trace_nu(4 * n, [(4 * st, c) for st, c in segs], passes=3, j0=j0)
        assert got.tolist() == want
        done += 1
    assert done > 100


def test_nonuniform_rejects_bad_segments(orc):
    with pytest.raises(ValueError):
        orc.trace_nu(64, [])                     # no segment
    with pytest.raises(ValueError):
        orc.trace_nu(64, [(4, 0)])               # empty segment
    with pytest.raises(ValueError):
        orc.trace_nu(64, [(6, 2)])               # stride not a multiple of elem
    with pytest.raises(ValueError):
        orc.trace_nu(64, [(4, 2)], j0=16)        # start outside the array


def test_nonuniform_revisit_breaks_lru_fifo_tie(orc):
    """Lines A, B, A, C, A in one fully associative 2-way set: LRU keeps A
    (the C miss evicts B) and hits the last access, FIFO evicts A (first in)
    and misses it.  Uniform chases cannot show this difference (Section 4.2
    step 4); a non-uniform chase that returns into a line can.  Elements
    0, 8, 1, 16, 2 with 32-byte lines are lines 0, 1, 0, 2, 0."""
    n = 64
    segs = [(4 * 8, 1), (4 * (n - 7), 1), (4 * 15, 1), (4 * (n - 14), 1), (4, 1)]
    idx = orc.trace_nu(4 * n, segs)
    assert idx.tolist() == [0, 8, 1, 16, 2]
    lru = orc.replay(orc.make_model(64, 32, 2, orc.LRU), idx)[0]
    fifo = orc.replay(orc.make_model(64, 32, 2, orc.FIFO), idx)[0]
    assert lru.tolist() == [0, 0, 1, 0, 1]
    assert fifo.tolist() == [0, 0, 1, 0, 0]


def test_nonuniform_section52_pattern(orc):
    """The Section 5.2 construction with s1 = 32 MB (65 accesses, then the
    same lines again three times) and s3 = one element (64 accesses from
    the start).  A fully associative LRU cache of 128 lines of 128 B keeps
    the 65 lines: 65 cold misses, 195 hits, then elements 0..31 hit (line
    0 is resident) and 32..63 are a new line: one miss, 31 hits.  With 64
    lines the 65-line loop thrashes: 260 misses; line 0 was evicted, so
    each of the two element lines misses once."""
    s1 = 32 << 20
    N = 65 * s1
    idx = orc.trace_nu(N, [(s1, 65 * 4), (4, 64)])
    assert idx[65] == 0 and idx[260] == 0 and idx[-1] == 63
    h128 = orc.replay(orc.make_model(128 * 128, 128, 128, orc.LRU), idx)[0]
    assert h128.tolist() == [0] * 65 + [1] * 195 + [1] * 32 + [0] + [1] * 31
    h64 = orc.replay(orc.make_model(64 * 128, 128, 64, orc.LRU), idx)[0]
    assert h64.tolist() == [0] * 260 + [0] + [1] * 31 + [0] + [1] * 31


# ---------------------------------------------------- I1: Fig. 3 --------
def test_fig3_worked_example(orc):
    """Section 4.1, Fig. 3: 12-word 2-way cache, 2-word lines, 3 sets, array
    of 13 words read one word at a time.  After the cold pass the pattern
    repeats with period 13 and the 1st, 7th and 13th elements miss."""
    m = orc.make_model(12 * 4, 2 * 4, 2, orc.LRU)
    assert m.sets == 3
    p = orc.make_probe(13 * 4, 4, passes=6)
    idx = orc.trace(p)
    hits, _, _ = orc.replay(m, idx)
    steady = hits[13:].reshape(-1, 13)
    assert (steady == steady[0]).all()           # periodic, period 13
    miss_elems = sorted(int(idx[13 + k]) + 1 for k in np.nonzero(steady[0] == 0)[0])
    assert miss_elems == [1, 7, 13]              # 1-based array elements


# ------------------------------------------- I2: N <= C never misses ----
@pytest.mark.parametrize("policy", [0, 1, 2, 3])
def test_fitting_array_has_no_steady_misses(orc, policy):
    """Section 4.2 step 1: C is the largest N at which every access hits."""
    rng = np.random.default_rng(7)
    for C, b, a in [(4096, 32, 4), (3 * 1024, 64, 2), (12288, 32, 96 // 8), (8192, 128, 64)]:
        if policy == orc.PLRU and a & (a - 1):
            continue
        m = orc.make_model(C, b, a, policy, seed=99)
        for _ in range(6):
            N = int(rng.integers(1, C // 4 + 1)) * 4
            s = int(rng.integers(1, 64)) * 4
            p = orc.make_probe(N, s, passes=3)
            idx = orc.trace(p)
            L = orc.cycle_len(p)
            hits, mt, ms = orc.replay(m, idx, count_from=L)
            assert ms == 0, (C, b, a, N, s)
            assert mt == len({(4 * j) // b for j in idx})   # one cold miss per line


# ----------------------------------- I3: Eq. (2) exact, Section 4.2 -----
@pytest.mark.parametrize("policy", [0, 1])
@pytest.mark.parametrize("C,b,a", [(4096, 32, 4), (12 * 1024, 32, 96), (16384, 128, 4),
                                   (3 * 2048, 64, 4), (8192, 64, 1)])
def test_overflow_by_lines_closed_form(orc, policy, C, b, a):
    """Section 4.2 step 3 / Eq. (2): with s dividing b and N a multiple of s,
    one steady pass misses exactly on every line of every set holding more
    than a lines: M(N) = sum_j n_j [n_j > a], n_j = #{l < ceil(N/b): l = j mod T}.
    At s = b and N = C + m*b this is m(a+1) misses per pass (Eq. (2) made
    exact)."""
    T = C // (a * b)
    model = orc.make_model(C, b, a, policy)
    for s in sorted({4, b // 2, b}):
        for N in list(range(C - 2 * b, C + (T + 2) * b + 1, s if s >= 32 else 32)):
            if N <= 0 or N % s:
                continue
            p = orc.make_probe(N, s, passes=2)
            L = orc.cycle_len(p)
            _, _, ms = orc.replay(model, orc.trace(p), count_from=L)
            nlines = -(-N // b)
            counts = [len(range(j, nlines, T)) for j in range(T)]
            expect = sum(n for n in counts if n > a)
            assert ms == expect, (s, N)
            if s == b and C < N <= C + T * b:
                assert ms == ((N - C) // b) * (a + 1)


# ---------------------- cyclic chases: closed forms per set, Section 4.1 --
def test_cyclic_chase_closed_forms(orc):
    """Two closed forms of the replay (the scoring kernels use both):
    (1) when every set holds at most a of the array's lines, any policy
    misses exactly on the first touch of each line; (2) LRU and FIFO on a
    chase whose every pass is one increasing sweep: each set's run starts
    (first access of each line visit) miss in the first pass, and in every
    later pass exactly when the set holds more lines than ways.  Random
    models with set_shift mappings, non-power-of-two sets and ways, j0 and
    base offsets, 1 to 3 passes."""
    rng = np.random.default_rng(5)
    checked = [0, 0]
    for _ in range(1500):
        b = int(rng.choice([4, 8, 16, 32]))
        a = int(rng.choice([1, 2, 3, 4, 8]))
        T = int(rng.choice([1, 2, 3, 4, 8]))
        pol = int(rng.choice([0, 1, 2, 3]))
        if pol == orc.PLRU and a & (a - 1):
            continue
        lb = b.bit_length() - 1
        ss = lb + int(rng.integers(0, 3)) if rng.random() < 0.3 else 0
        C = a * b * T
        N = int(rng.integers(1, 6 * C // 4 + 2)) * 4
        s = int(rng.integers(1, 3 * b // 4 + 2)) * 4
        passes = int(rng.integers(1, 4))
        j0 = int(rng.integers(0, N // 4)) if rng.random() < 0.3 else 0
        base = int(rng.integers(0, 64)) * 4 if rng.random() < 0.3 else 0
        m = orc.make_model(C, b, a, pol, set_shift=ss, seed=7)
        p = orc.make_probe(N, s, passes=passes, j0=j0, base=base)
        idx = np.asarray(orc.trace(p), np.int64)
        L = orc.cycle_len(p)
        hits, _, _ = orc.replay(m, idx, base=base, trace_id=3, count_from=0)
        miss = 1 - np.asarray(hits)
        addr = base + 4 * idx
        us = ss if ss else lb
        sets, lines = (addr >> us) % T, addr >> lb
        units = ((base + (N // 4 - 1) * 4) >> us) - (base >> us) + 1
        if (-(-units // T)) << (us - lb) <= a:
            first = np.zeros(len(idx), np.uint8)
            first[np.unique(lines, return_index=True)[1]] = 1
            assert np.array_equal(miss, first), (C, b, a, pol, ss, N, s, passes, j0, base)
            checked[0] += 1
        ne, se = N // 4, (s // 4) % (N // 4)
        if pol in (orc.LRU, orc.FIFO) and (se == 0 or (ne - j0 + se - 1) // se >= L):
            expect = np.zeros(len(idx), np.uint8)
            for t in range(T):
                ks = np.nonzero(sets[:L] == t)[0]
                starts = [k for i, k in enumerate(ks) if i == 0 or lines[k] != lines[ks[i - 1]]]
                n_lines = len({int(lines[k]) for k in ks})
                for q in range(passes if n_lines > a else 1):
                    expect[np.asarray(starts, np.int64) + q * L] = 1
            assert np.array_equal(miss, expect), (C, b, a, pol, ss, N, s, passes, j0, base)
            checked[1] += 1
    assert min(checked) > 100, checked


def test_plru_cyclic_pattern_depends_only_on_ways_and_lines(orc):
    """Tree-PLRU on a chase whose pass is one increasing sweep: each set
    sees its n lines in the same cyclic order every pass, so (the policy
    being deterministic and blind to line identities) the set's hit/miss
    sequence depends only on (a, n).  Checked across sets of one model, and
    across models with different capacities, line sizes, set counts and
    strides (the scoring kernels tabulate one pattern per (a, n))."""
    seen = {}
    checked = 0
    for a in (4, 8, 16):
        for T in (1, 2, 3, 5, 8):
            for b in (16, 32, 64):
                C = a * b * T
                for s in (b // 2, b, 2 * b):
                    for N in (C + b * (T // 2 + 1), C + 3 * b * T + 4 * b, 2 * C - 2 * s):
                        N -= N % s
                        p = orc.make_probe(N, s, passes=2)
                        idx = np.asarray(orc.trace(p), np.int64)
                        L = orc.cycle_len(p)
                        ne, se = N // 4, (s // 4) % (N // 4)
                        if not (se == 0 or (ne + se - 1) // se >= L):
                            continue
                        hits, _, _ = orc.replay(orc.make_model(C, b, a, orc.PLRU), idx)
                        hits = np.asarray(hits)
                        lines = (4 * idx) // b
                        for t in range(T):
                            ks = np.nonzero(lines[:L] % T == t)[0]
                            starts = [k for i, k in enumerate(ks) if i == 0 or lines[k] != lines[ks[i - 1]]]
                            n = len(starts)
                            pat = tuple(int(hits[k + L]) for k in starts)
                            assert seen.setdefault((a, n), pat) == pat, (a, n, C, b, T, N, s)
                            checked += 1
    assert checked > 300 and len(seen) > 20
    # not trivial: some pattern has hits and misses beyond the first pass
    assert any(0 < sum(p) < len(p) for (a, n), p in seen.items() if n > a)


# ------------------------------------ I4: Eq. (1), Section 4.1 ---------
@pytest.mark.parametrize("C,b,a", [(4096, 32, 4), (16384, 64, 8), (8192, 128, 2), (32768, 32, 16)])
def test_eq1_stride_special_cases(orc, C, b, a):
    """Eq. (1), N >> C with N and s powers of two: the miss rate is s/b for
    s < b, 1 while N/s exceeds a, and 0 once the N/s lines fit the ways."""
    model = orc.make_model(C, b, a, orc.LRU)
    for N in (2 * C, 4 * C):
        s = 4
        while s <= N:
            p = orc.make_probe(N, s, passes=2)
            L = orc.cycle_len(p)
            _, _, ms = orc.replay(model, orc.trace(p), count_from=L)
            r = Fraction(ms, L)
            if s < b:
                assert r == Fraction(s, b), (N, s)
            elif N // s > a:
                assert r == 1, (N, s)
            else:
                assert r == 0, (N, s)
            s *= 2


# --------------------------------------- I5: policy equivalences --------
def _random_trace(rng, n, span):
    return rng.integers(0, span, size=n).astype(np.int32)


def test_policy_equivalences(orc):
    """One way: every policy is the same cache.  Two ways: tree-PLRU is LRU.
    Uniform-stride chases whose pass is one increasing sweep (s divides N)
    visit each set's lines in the same cyclic order every pass, so they
    cannot tell LRU from FIFO (Section 4.2 step 4 needs the per-access trace
    for that); random traces can."""
    rng = np.random.default_rng(11)
    differ = 0
    for t in range(60):
        idx = _random_trace(rng, 300, 400)
        for C, b in [(1024, 32), (2048, 64)]:
            outs = [orc.replay(orc.make_model(C, b, 1, pol, seed=t), idx, trace_id=t)[0]
                    for pol in range(4)]
            assert all((o == outs[0]).all() for o in outs)
            lru2 = orc.replay(orc.make_model(C, b, 2, orc.LRU), idx)[0]
            plru2 = orc.replay(orc.make_model(C, b, 2, orc.PLRU), idx)[0]
            assert (lru2 == plru2).all()
            lru4 = orc.replay(orc.make_model(C, b, 4, orc.LRU), idx)[0]
            fifo4 = orc.replay(orc.make_model(C, b, 4, orc.FIFO), idx)[0]
            differ += int((lru4 != fifo4).any())
    assert differ > 0
    for N in range(3000, 9000, 388):
        for s in (4, 32, 64, 96, 256):
            p = orc.make_probe(N - N % s, s, passes=3)
            idx = orc.trace(p)
            for a in (2, 4, 8):
                h1 = orc.replay(orc.make_model(4096, 32, a, orc.LRU), idx)[0]
                h2 = orc.replay(orc.make_model(4096, 32, a, orc.FIFO), idx)[0]
                assert (h1 == h2).all()


# ----------------------------- I6: Fig. 11 LRU counterfactual ------------
def test_fig11_one_line_overflow_thrashes_one_set(orc):
    """Section 4.5 / Fig. 11: overflowing a 16 KB, 128 B-line, 4-way cache by
    one line (N = 16.125 KB, s = 128 B) leaves every miss in one set, and
    under LRU every access to that set misses (a+1 per pass)."""
    model = orc.make_model(16384, 128, 4, orc.LRU)
    p = orc.make_probe(16384 + 128, 128, passes=8)
    idx = orc.trace(p)
    L = orc.cycle_len(p)
    hits, _, ms = orc.replay(model, idx, count_from=L)
    miss_lines = {int(idx[k]) * 4 // 128 for k in range(L, len(idx)) if hits[k] == 0}
    assert ms == 7 * 5 and miss_lines == {0, 32, 64, 96, 128}
    # a non-LRU policy turns some of those accesses into hits
    plru = orc.make_model(16384, 128, 4, orc.PLRU)
    _, _, ms_p = orc.replay(plru, idx, count_from=L)
    assert 0 < ms_p < ms


# ----------------------------------- I7: brute force on tiny caches -----
SMALL = [(T, a) for T in range(1, 9) for a in range(1, 9) if T * a <= 8]


@pytest.mark.parametrize("policy", [0, 1, 2, 3])
def test_brute_force_tiny_caches(orc, policy):
    rng = np.random.default_rng(100 + policy)
    for T, a in SMALL:
        if policy == 2 and (a & (a - 1)):
            continue
        for b in (4, 8):
            for shift in (0, 4) if b == 4 else (0,):
                model = orc.make_model(T * a * b, b, a, policy, set_shift=shift, seed=12345)
                for trial in range(25):
                    n = int(rng.integers(1, 40))
                    idx = _random_trace(rng, n, int(rng.integers(1, 3 * T * a * b // 4 + 2)))
                    base = int(rng.integers(0, 4)) * 4
                    got, mt, _ = orc.replay(model, idx, base=base, trace_id=trial)
                    exp = brute.hits_for(policy, idx.tolist(), b, a, T, seed=12345,
                                         trace_id=trial, base=base, set_shift=shift)
                    assert got.tolist() == exp, (T, a, b, shift, idx.tolist())
                    assert mt == len(idx) - sum(exp)


def test_brute_force_exhaustive_short_traces(orc):
    """Every trace of length 6 over 4 lines, every tiny (T, a), every policy."""
    import itertools
    for T, a in [(1, 1), (1, 2), (2, 1), (1, 4), (2, 2), (4, 2), (1, 8), (2, 4)]:
        for pol in range(4):
            model = orc.make_model(T * a * 4, 4, a, pol, seed=3)
            for tr in itertools.product(range(4), repeat=6):
                idx = np.array(tr, dtype=np.int32)
                got = orc.replay(model, idx)[0].tolist()
                assert got == brute.hits_for(pol, list(tr), 4, a, T, seed=3)


def test_lru_inclusion_property(orc):
    """LRU is a stack algorithm: with b and T fixed, hits at a are hits at a+1."""
    rng = np.random.default_rng(5)
    for _ in range(40):
        idx = _random_trace(rng, 400, 700)
        prev = None
        for a in range(1, 10):
            h = orc.replay(orc.make_model(4 * 32 * a, 32, a, orc.LRU, T=4), idx)[0]
            if prev is not None:
                assert (prev <= h).all()
            prev = h


def test_random_policy_depends_only_on_counter(orc):
    """RANDOM draws from Philox keyed by (access index, trace id): the same
    key and counter give the same trace, another trace id another one."""
    rng = np.random.default_rng(9)
    idx = _random_trace(rng, 2000, 600)
    m = orc.make_model(1024, 32, 8, orc.RANDOM, seed=0xABCDEF0123)
    h1 = orc.replay(m, idx, trace_id=5)[0]
    h2 = orc.replay(m, idx, trace_id=5)[0]
    h3 = orc.replay(m, idx, trace_id=6)[0]
    assert (h1 == h2).all() and (h1 != h3).any()


# ------------------------------------------------------------ Philox -----
def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    for ctr, key, out in _kat():
        assert orc.philox(ctr, key).tolist() == out
        assert brute.philox4x32_10(ctr, key) == out


def test_philox_matches_rocrand(orc, tmp_path):
    """Cross-check against rocRAND's Philox4x32-10, compiled for the host."""
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers or g++ not available")
    exe = tmp_path / "philox_rocrand"
    subprocess.check_call([gxx, "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           os.path.join(HERE, "native", "philox_rocrand.cpp"), "-o", str(exe)])
    rng = np.random.default_rng(31337)
    rows = rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64)
    text = "\n".join(" ".join(f"{int(v):08x}" for v in r) for r in rows) + "\n"
    res = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True)
    lines = res.stdout.split("\n")
    for r, line in zip(rows, lines):
        want = [int(x, 16) for x in line.split()]
        assert orc.philox(r[:4], r[4:]).tolist() == want


# ----------------------------------------------------- classification ----
def test_latency_threshold_two_levels(orc):
    """Section 4.1 model t = t0 + tm*r with two latency populations; levels
    from Section 5.2 (GTX780: 198 cycles cache hit, 339 cycles L1 TLB hit /
    cache miss)."""
    rng = np.random.default_rng(3)
    truth = rng.integers(0, 2, size=5000).astype(np.uint8)
    lat = np.where(truth == 1, 198 + rng.integers(0, 12, size=5000),
                   339 + rng.integers(0, 30, size=5000)).astype(np.uint32)
    theta = orc.auto_threshold(lat)
    assert 198 <= theta < 339
    assert (orc.classify(lat, theta) == truth).all()
    assert orc.auto_threshold(np.array([5, 5, 5], dtype=np.uint32)) == 5


# ----------------------------------------------------------- inference ---
def test_inference_recovers_target(orc):
    """Section 4.2 / Fig. 6: the observed cache reproduces its own traces,
    so it is in the zero-mismatch class, and the reported best is the lowest
    canonical index with the exact minimum of m/n."""
    from paper_1509_02308_amd import workloads as W
    cands = W.candidate_grid(Cs=(4096, 6144, 8192), bs=(32, 64), As=(1, 2, 4, 8),
                             policies=(0, 1, 2))
    om = [orc.make_model(int(c["C"]), int(c["b"]), int(c["a"]), int(c["policy"])) for c in cands]
    probes = W.sweep_union(cands)
    op = [orc.make_probe(int(p["N"]), int(p["s"]), int(p["passes"])) for p in probes]
    for target in (0, 7, len(om) - 1):
        obs, off, cf = [], [], []
        pos = 0
        for i, p in enumerate(op):
            idx = orc.trace(p)
            h, _, _ = orc.replay(om[target], idx, trace_id=i)
            obs.append(h)
            off.append(pos)
            cf.append(orc.cycle_len(p))
            pos += len(h)
        best, m, n = orc.infer(om, op, np.concatenate(obs), off, cf, probe_select=1)
        assert m[target] == 0
        ratios = [Fraction(int(mi), int(ni)) if ni else None for mi, ni in zip(m, n)]
        lo = min(r for r in ratios if r is not None)
        assert best == min(i for i, r in enumerate(ratios) if r == lo)
        assert ratios[best] == 0
        # n counts the compared (second-pass) accesses of the candidate's own sweep
        for c in range(len(om)):
            own = [i for i, p in enumerate(op) if orc.in_own_sweep(om[c], p)]
            assert int(n[c]) == sum(orc.cycle_len(op[i]) for i in own)
