"""Pins of the adaptive probe planner (oracle/planner.py): the two-stage
procedure of Sec. 4.2 (Fig. 6) as a greedy choice among pool probes.  The
choice rule (smallest largest class, then most classes, then lowest index)
is this build's; what it must satisfy is pinned here against the C
oracle's exhaustive inference, brute-force replays and the capacity step of
Fig. 6."""
import numpy as np
import pytest

from oracle import brute
from oracle import planner as P

CANDS = [(C, 32, a, pol) for C in (4096, 8192, 12288, 16384) for a in (2, 4) for pol in (0, 1, 2)]
POOL = [(N, s, 2) for N in range(2048, 24577, 2048) for s in (4, 32, 64)]


def _observation(orc, target, pool):
    hits, off, cf = [], [0], []
    for N, s, passes in pool:
        pr = orc.make_probe(N, s, passes=passes)
        h, _, _ = orc.replay(orc.make_model(*target[:4]), orc.trace(pr))
        hits.append(h)
        off.append(off[-1] + len(h))
        cf.append(orc.cycle_len(pr))
    return np.concatenate(hits), np.array(off[:-1], np.uint64), np.array(cf, np.uint64)


@pytest.mark.parametrize("target", range(0, len(CANDS), 3))
def test_adaptive_ends_at_the_exhaustive_zero_class(orc, target):
    """Whatever probes it picks, the loop keeps exactly the candidates that
    reproduce the target on every pool probe (steady passes): the zero class
    of the exhaustive search over the whole pool."""
    surv, used = P.adaptive(orc, CANDS, POOL, CANDS[target])
    obs, off, cf = _observation(orc, CANDS[target], POOL)
    cands = [orc.make_model(*c) for c in CANDS]
    probes = [orc.make_probe(*p) for p in POOL]
    _, m, _ = orc.infer(cands, probes, obs, off, cf, probe_select=0)
    assert surv == orc.zero_class(m).tolist()
    assert target in surv
    assert len(used) < len(POOL)


def test_each_probe_splits_the_survivors(orc):
    cls = P.classes(orc, CANDS, POOL)
    for target in range(len(CANDS)):
        alive = np.ones(len(CANDS), dtype=bool)
        while True:
            p, worst, n = P.next_probe(cls, alive)
            if worst >= alive.sum():
                # no probe splits them: every probe puts them in one class
                assert all(len(set(cls[q][alive])) == 1 for q in range(len(POOL)))
                break
            assert n >= 2
            keep = cls[p] == cls[p][target]
            assert 0 < (alive & keep).sum() < alive.sum()
            alive &= keep
            assert alive[target]


def test_classes_match_brute_force(orc):
    """Class = lowest candidate with the same steady bits, the bits taken
    from the brute-force replays."""
    cands = [(512, 16, a, pol) for a in (1, 2, 4) for pol in (0, 1, 2)] + [(768, 16, 3, 0), (768, 16, 3, 1)]
    pool = [(N, s, 2) for N in (256, 512, 640, 768, 1024) for s in (4, 16, 48)]
    cls = P.classes(orc, cands, pool)
    for p, (N, s, passes) in enumerate(pool):
        n, se = N // 4, s // 4
        L = n // np.gcd(n, se % n)
        idx = brute.listing_trace(n, se, passes * L)
        sig = [tuple(brute.hits_for(pol, idx, b, a, C // (a * b))[L:]) for C, b, a, pol in cands]
        want = [sig.index(x) for x in sig]
        assert cls[p].tolist() == want


def test_capacity_step_of_fig6(orc):
    """Fig. 6 step 1 (s = one element, N ramping): on an LRU target with
    C >= N every access of the probe hits, and only the candidates with
    C >= N predict that, so one observation keeps exactly them."""
    cands = [(C, 32, 4, 0) for C in (4096, 8192, 12288, 16384, 20480)]
    pool = [(N, 4, 2) for N in (4096, 8192, 12288, 16384, 20480)]
    cls = P.classes(orc, cands, pool)
    for p, (N, _, _) in enumerate(pool):
        for t, (Ct, _, _, _) in enumerate(cands):
            if Ct >= N:
                survivors = [c for c in range(len(cands)) if cls[p][c] == cls[p][t]]
                assert survivors == [c for c, (C, _, _, _) in enumerate(cands) if C >= N]
