"""Pins of the generalised cache replay (per-set associativity, set tables,
weighted random replacement) against brute force, special cases, closed
forms and the replacement probabilities the paper reports.

Passages: Sec. 4.3 (texture L1: set chosen by address bits 7-8), Sec. 4.4 and
Fig. 9 (L2 TLB: one set of 17 entries and six of 8), Sec. 4.5 (Fermi L1:
way 2 replaced with probability 1/2, the other ways 1/6)."""
import numpy as np
import pytest

from oracle import brute


def test_general_matches_brute_force(orc):
    rng = np.random.default_rng(3)
    for t in range(400):
        T = int(rng.integers(1, 6))
        pol = int(rng.integers(0, 5))
        ways = [int(2 ** rng.integers(0, 4)) if pol == 2 else int(rng.integers(1, 9)) for _ in range(T)]
        table = [int(x) for x in rng.integers(0, T, size=int(rng.integers(1, 9)))] if rng.random() < 0.5 else None
        weights = [int(x) for x in rng.integers(0, 5, size=max(ways))]
        weights[0] += 1
        b = int(2 ** rng.integers(2, 6))
        sh = int(np.log2(b)) + int(rng.integers(0, 3)) if rng.random() < 0.3 else 0
        idx = rng.integers(0, 300, size=200).astype(np.int32)
        seed = int(rng.integers(0, 2 ** 40))
        g = orc.General(b, ways, pol, sh, table, weights if pol == 4 else None, seed)
        got = orc.replay_general(g, idx, trace_id=t)[0].tolist()
        assert got == brute.general_hits(pol, idx.tolist(), b, ways, table, weights, seed, t, set_shift=sh)


@pytest.mark.parametrize("policy", [0, 1, 2, 3])
def test_equal_sets_without_table_is_the_standard_model(orc, policy):
    rng = np.random.default_rng(10 + policy)
    for t in range(40):
        a = int(2 ** rng.integers(0, 4))
        T = int(rng.integers(1, 9))
        b = 32
        idx = rng.integers(0, 2000, size=500).astype(np.int32)
        std = orc.replay(orc.make_model(T * a * b, b, a, policy, seed=t + 1), idx, trace_id=t, count_from=100)
        gen = orc.replay_general(orc.General(b, [a] * T, policy, seed=t + 1), idx, trace_id=t, count_from=100)
        assert std[0].tolist() == gen[0].tolist() and std[1:] == gen[1:]


def test_unit_weights_are_uniform_random(orc):
    """u mod a picks way u mod a either way."""
    rng = np.random.default_rng(4)
    for t in range(40):
        a = int(rng.integers(1, 9))
        idx = rng.integers(0, 3000, size=400).astype(np.int32)
        r = orc.replay_general(orc.General(32, [a] * 3, orc.RANDOM, seed=99), idx, trace_id=t)[0]
        w = orc.replay_general(orc.General(32, [a] * 3, orc.WRANDOM, weights=[1] * a, seed=99), idx, trace_id=t)[0]
        assert r.tolist() == w.tolist()


@pytest.mark.parametrize("policy", [0, 1, 2, 3, 4])
def test_set_table_identity_and_relabelling(orc, policy):
    """A table 0..T-1 is the modulo mapping; with equal sets, permuting the
    table only renames sets, which changes no hit."""
    rng = np.random.default_rng(20 + policy)
    T, a = 4, 4
    for t in range(20):
        idx = rng.integers(0, 4000, size=600).astype(np.int32)
        kw = dict(weights=[1, 3, 1, 1], seed=7) if policy == 4 else dict(seed=7)
        base = orc.replay_general(orc.General(32, [a] * T, policy, **kw), idx, trace_id=t)[0]
        ident = orc.replay_general(orc.General(32, [a] * T, policy, table=list(range(T)), **kw), idx, trace_id=t)[0]
        perm = orc.replay_general(orc.General(32, [a] * T, policy, table=[2, 0, 3, 1], **kw), idx, trace_id=t)[0]
        assert base.tolist() == ident.tolist() == perm.tolist()


def _steady_misses(orc, g, n_lines, b):
    idx = orc.trace(orc.make_probe(n_lines * b, b, passes=3))
    _, _, ms = orc.replay_general(g, idx, count_from=n_lines)
    return ms // 2          # per pass


def test_unequal_sets_lru_closed_form(orc):
    """A chase over n lines, one access per line, visits set t's m_t lines
    cyclically: under LRU a set misses all of them each pass if m_t exceeds
    its ways and none otherwise."""
    rng = np.random.default_rng(6)
    for _ in range(30):
        T = int(rng.integers(1, 8))
        ways = [int(x) for x in rng.integers(1, 20, size=T)]
        n = int(rng.integers(1, 3 * sum(ways)))
        m = [len(range(t, n, T)) for t in range(T)]
        want = sum(mt for mt, w in zip(m, ways) if mt > w)
        assert _steady_misses(orc, orc.General(64, ways, orc.LRU), n, 64) == want


def test_l2_tlb_staircase(orc):
    """Sec. 4.4 / Fig. 9: 2 MB entries in one set of 17 ways and six of 8 (65
    entries).  With a 65-entry table that gives the large set 17 residues and
    each small set 8, residues 0..6 landing on sets 0..6, a chase at s = 2 MB
    fits up to 130 MB; the next page overflows the large set, and each page
    after it overflows one more small set: the steady misses rise in one step
    of 17 + 1 and then in steps of 8 + 1, the piecewise-linear shape the paper
    measures (it counts the set's entries, 17 and 8)."""
    page = 2 << 20
    table = [r % 7 for r in range(56)] + [0] * 9
    assert [table.count(t) for t in range(7)] == [17, 8, 8, 8, 8, 8, 8]
    g = orc.General(page, [17] + [8] * 6, orc.LRU, table=table)
    steps = [_steady_misses(orc, g, n, page) for n in range(64, 72)]
    assert steps == [0, 0, 18, 27, 36, 45, 54, 63]


def test_weighted_random_victim_probabilities(orc):
    """Sec. 4.5: weights (1, 3, 1, 1) give way 2 (index 1) probability 1/2 and
    the others 1/6.  Lines A, B, C, D fill ways 0-3 of a 4-way set, E evicts
    one of them, and a last access to X in {A, B, C, D} misses iff X's way was
    the victim.  The four traces differ only after the draw, so exactly one
    of the four last accesses misses in each trial."""
    g = orc.General(32, [4], orc.WRANDOM, weights=[1, 3, 1, 1], seed=1509)
    lines = [0, 8, 16, 24, 32]                    # elements of lines A..E (32 B lines)
    n = 6000
    miss = np.zeros((n, 4), dtype=np.int64)
    for t in range(n):
        for x in range(4):
            idx = np.array(lines + [lines[x]], np.int32)
            miss[t, x] = 1 - int(orc.replay_general(g, idx, trace_id=t)[0][-1])
    assert (miss.sum(axis=1) == 1).all()
    frac = miss.mean(axis=0)
    for f, p in zip(frac, [1 / 6, 1 / 2, 1 / 6, 1 / 6]):
        assert abs(f - p) < 5 * np.sqrt(p * (1 - p) / n)


def _one_line_overflow_miss_rate(p):
    """Exact stationary miss rate of a 4-way set under weighted random
    replacement with a cyclic reference string over 5 lines (Fig. 11: the
    cache overflowed by one line), by power iteration over (line in each way,
    next line) states."""
    from itertools import permutations
    states = [(perm, nxt) for perm in permutations(range(5), 4) for nxt in range(5)]
    index = {s: i for i, s in enumerate(states)}
    P = np.zeros((len(states), len(states)))
    miss = np.zeros(len(states))
    for (perm, nxt), i in index.items():
        after = (nxt + 1) % 5
        if nxt in perm:
            P[i, index[(perm, after)]] += 1.0
        else:
            miss[i] = 1.0
            for w in range(4):
                q = list(perm)
                q[w] = nxt
                P[i, index[(tuple(q), after)]] += p[w]
    pi = np.full(len(states), 1.0 / len(states))
    for _ in range(5000):
        pi = pi @ P
    return float(pi @ miss)


def test_weighted_random_one_line_overflow_rate(orc):
    """Sec. 4.5 / Fig. 11: with one line too many, LRU misses every access; the
    weighted random policy hits some, at the rate its Markov chain fixes."""
    p = [1 / 6, 1 / 2, 1 / 6, 1 / 6]
    want = _one_line_overflow_miss_rate(p)
    assert 0.3 < want < 1.0
    passes = 40000
    idx = orc.trace(orc.make_probe(5 * 32, 32, passes=passes))
    _, _, ms = orc.replay_general(orc.General(32, [4], orc.WRANDOM, weights=[1, 3, 1, 1], seed=11), idx,
                                  count_from=50)
    rate = ms / (len(idx) - 50)
    assert abs(rate - want) < 0.01
    _, _, ms_lru = orc.replay_general(orc.General(32, [4], orc.LRU), idx, count_from=50)
    assert ms_lru == len(idx) - 50


def test_general_rejects_bad_models(orc):
    assert not orc.General(48, [4], orc.LRU).ok()                    # line not a power of two
    assert not orc.General(32, [4, 0], orc.LRU).ok()                 # empty set
    assert not orc.General(32, [4, 3], orc.PLRU).ok()                # PLRU needs 2^k ways
    assert not orc.General(32, [4], orc.LRU, table=[0, 1]).ok()      # table entry outside the sets
    assert not orc.General(32, [4], orc.WRANDOM).ok()                # weights missing
    assert not orc.General(32, [2], orc.WRANDOM, weights=[0, 0]).ok()  # zero total weight
    assert not orc.General(64, [4], orc.LRU, set_shift=5).ok()       # set unit smaller than a line


# ------------------------------------------------ generalised inference ---
def _general(orc, d):
    return orc.General(d["line"], d["ways"], d.get("policy", 0), d.get("set_shift", 0), d.get("table"),
                       d.get("weights"), d.get("seed", 0))


def _brute_hits(d, idx, trace_id):
    return brute.general_hits(d.get("policy", 0), idx.tolist(), d["line"], d["ways"], d.get("table"),
                              d.get("weights"), d.get("seed", 0), trace_id, set_shift=d.get("set_shift", 0))


def _observe(orc, target, rows):
    """Hit bytes of the target on each probe (trace id = probe index, as the
    inference replays them), offsets and the first compared access."""
    g = _general(orc, target)
    hits, off, cf = [], [0], []
    for i, r in enumerate(rows):
        p = orc.make_probe(*r)
        h, _, _ = orc.replay_general(g, orc.trace(p), trace_id=i)
        hits.append(h)
        off.append(off[-1] + len(h))
        cf.append(orc.cycle_len(p))
    return np.concatenate(hits), np.array(off[:-1], np.uint64), np.array(cf, np.uint64)


def test_infer_general_counts_match_brute_force(orc):
    """m[c] = the accesses from the first steady one on whose hit differs from
    the observation, summed over probes, each candidate replayed by the
    per-set brute force; n[c] the accesses compared."""
    from paper_1509_02308_amd import workloads as W
    cands = [d for d in W.random_general(12, seed=31) if sum(d["ways"]) * d["line"] <= 4096]
    assert len(cands) >= 4
    rows = [(N, s, 2) for N, s in ((256, 16), (512, 32), (640, 64), (1024, 128), (96, 4))]
    target = cands[1]
    obs, off, cf = _observe(orc, target, rows)
    best, m, n = orc.infer_general([_general(orc, d) for d in cands], [orc.make_probe(*r) for r in rows], obs, off, cf)
    for c, d in enumerate(cands):
        mm = nn = 0
        for p, r in enumerate(rows):
            tr = orc.trace(orc.make_probe(*r))
            h = np.array(_brute_hits(d, tr, p), np.uint8)
            o = obs[int(off[p]):int(off[p]) + len(tr)]
            mm += int((h[int(cf[p]):] != o[int(cf[p]):]).sum())
            nn += len(tr) - int(cf[p])
        assert (int(m[c]), int(n[c])) == (mm, nn), (c, d)
    assert m[1] == 0 and best == int(np.nonzero(m == 0)[0][0])


@pytest.mark.parametrize("name", ["texture_l1", "readonly_table", "l2_tlb", "fermi_l1"])
def test_infer_general_recovers_paper_shaped_targets(orc, name):
    """Sections 4.3-4.5: around each paper-shaped target (texture L1 set
    bits, read-only table mapping, the L2 TLB's 17 + 6 x 8 staircase of
    Fig. 9, Fermi's weighted replacement) a family of neighbours; the
    candidates that reproduce the target's hits exactly (found by brute
    force) are the zero class, the target is among them and the best is the
    first of them."""
    from paper_1509_02308_amd import workloads as W
    target = [t for t in W.paper_general_targets() if t["name"] == name][0]
    fam, at = W.general_family(target)
    rows = W.general_probe_rows(target)
    if name == "readonly_table":
        # tables differ only where a set overflows: line strides just past
        # the capacity; the neighbours with the target's mapping unit
        C = 32 * sum(target["ways"])
        rows = [r for r in rows if r[1] == 32 and C <= r[0] <= C + 1024]
        keep = [c for c, d in enumerate(fam) if d["set_shift"] == target["set_shift"]]
        at = keep.index(at)
        fam = [fam[c] for c in keep]
    else:
        # short traces keep the brute force quick
        rows = [r for r in rows if r[0] // r[1] <= 160]
        rows = [rows[i] for i in np.linspace(0, len(rows) - 1, 8).astype(int)]
    obs, off, cf = _observe(orc, target, rows)
    best, m, n = orc.infer_general([_general(orc, d) for d in fam], [orc.make_probe(*r) for r in rows], obs, off, cf)
    brute_zero = []
    for c, d in enumerate(fam):
        same = True
        for p, r in enumerate(rows):
            tr = orc.trace(orc.make_probe(*r))
            h = np.array(_brute_hits(d, tr, p), np.uint8)
            o = obs[int(off[p]):int(off[p]) + len(tr)]
            if not np.array_equal(h[int(cf[p]):], o[int(cf[p]):]):
                same = False
                break
        if same:
            brute_zero.append(c)
    assert at in brute_zero
    assert np.nonzero(m == 0)[0].tolist() == brute_zero
    assert best == brute_zero[0]
    assert len(brute_zero) < len(fam)          # the probes separate the family
