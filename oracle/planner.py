"""Adaptive probe planning: the two-stage procedure of Sec. 4.2 (Fig. 6)
generalised to a greedy choice among a pool of (N, s) probes.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

The paper picks each next (N, s) from what the previous runs showed: s = one
element and N ramping to find C, then b, then s = b to count sets, then a
long run for the policy.  Here the candidates that still agree with every
observation so far are the survivors; a probe splits them into classes of
candidates that predict the same steady-pass hit bits on it (accesses L ..
len-1, the first pass warming the cache); the next probe is the one whose
largest class among the survivors is smallest, then the one with more
classes, then the lowest pool index.  Observing the target on that probe
keeps the survivors of the target's class.  When no probe splits the
survivors any more they are indistinguishable on the pool.
"""
from __future__ import annotations

import numpy as np


def steady_bits(orc, model_row, probe_row) -> bytes:
    """Steady-pass hit bits of one (model, probe), as bytes."""
    C, b, a, pol = [int(x) for x in model_row[:4]]
    sh = int(model_row[4]) if len(model_row) > 4 else 0
    seed = int(model_row[5]) if len(model_row) > 5 else 0
    N, s, passes = [int(x) for x in probe_row[:3]]
    pr = orc.make_probe(N, s, passes=passes)
    L = orc.cycle_len(pr)
    hits, _, _ = orc.replay(orc.make_model(C, b, a, pol, set_shift=sh, seed=seed), orc.trace(pr), count_from=L)
    return bytes(hits[L:])


def classes(orc, cands, pool) -> np.ndarray:
    """cls[p, c] = lowest candidate index with the same steady bits as c on
    probe p."""
    cls = np.zeros((len(pool), len(cands)), dtype=np.int64)
    for p, pr in enumerate(pool):
        first = {}
        for c, m in enumerate(cands):
            cls[p, c] = first.setdefault(steady_bits(orc, m, pr), c)
    return cls


def score(cls_row, alive) -> tuple:
    """(largest class, number of classes) among the alive candidates."""
    sizes = {}
    for c in np.nonzero(alive)[0]:
        sizes[cls_row[c]] = sizes.get(cls_row[c], 0) + 1
    return (max(sizes.values()) if sizes else 0, len(sizes))


def next_probe(cls, alive):
    """(probe, largest class, number of classes) of the pool's best split."""
    best = None
    for p in range(cls.shape[0]):
        worst, n = score(cls[p], alive)
        key = (worst, -n, p)
        if best is None or key < best[0]:
            best = (key, p, worst, n)
    return best[1], best[2], best[3]


def adaptive(orc, cands, pool, target_row, max_steps=None):
    """Runs the loop against a target cache (observations are its replays).
    Returns (survivor indices, probes used in order)."""
    cls = classes(orc, cands, pool)
    alive = np.ones(len(cands), dtype=bool)
    used = []
    for _ in range(max_steps or len(pool)):
        p, worst, _ = next_probe(cls, alive)
        if worst >= int(alive.sum()):
            break
        obs = steady_bits(orc, target_row, pool[p])
        keep = np.array([steady_bits(orc, m, pool[p]) == obs for m in cands])
        alive &= keep
        used.append(p)
    return np.nonzero(alive)[0].tolist(), used
