"""GPU parity of the adaptive probe planner (Sec. 4.2, Fig. 6 as a greedy
split): class matrix, choices for seeded survivor sets and the whole loop
(choose, observe the target, keep its zero class) against oracle/planner.py."""
import numpy as np
import pytest

import oracle as orc
from oracle import planner as P
from paper_1509_02308_amd import workloads as W
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu

SMALL_CANDS = [(C, 32, a, pol) for C in (4096, 8192, 12288, 16384) for a in (2, 4) for pol in (0, 1, 2)]
SMALL_POOL = [(N, s, 2) for N in range(2048, 24577, 2048) for s in (4, 32, 64)]


def _grid():
    cands = [(int(c["C"]), int(c["b"]), int(c["a"]), int(c["policy"])) for c in W.candidate_grid()]
    pool = [(4096 + 2048 * i, s, 2) for i in range(32) for s in (32, 128)]
    return cands, pool


def _bitmap(mask):
    words = np.zeros((len(mask) + 31) // 32, dtype=np.uint32)
    for c in np.nonzero(mask)[0]:
        words[c // 32] |= np.uint32(1 << (c % 32))
    return words


@pytest.mark.parametrize("which", ["small", "grid"])
def test_planner_classes_and_choices_match_oracle(which):
    torch, capi = need_gpu()
    cands, pool = (SMALL_CANDS, SMALL_POOL) if which == "small" else _grid()
    carr, parr = capi.models(cands), capi.probes(pool)
    cls = torch.full((len(pool) * len(cands),), -1, dtype=torch.int32, device="cuda")
    alive = np.ones(len(cands), dtype=bool)
    say(f"pchase_plan_next_probe {which}: {len(cands)} candidates x {len(pool)} probes")
    ch = capi.pchase_plan_next_probe(carr, parr, _bitmap(alive), cls)
    want = P.classes(orc, cands, pool)
    assert np.array_equal(cls.cpu().numpy().reshape(len(pool), len(cands)), want)
    rng = np.random.default_rng(31)
    masks = [alive] + [rng.random(len(cands)) < f for f in (0.5, 0.2, 0.05, 0.01)] + [np.eye(len(cands), dtype=bool)[3]]
    for i, m in enumerate(masks):
        if i:
            say(f"  survivors {int(m.sum())}")
            ch = capi.pchase_plan_next_probe(carr, parr, _bitmap(m))
        p, worst, n = P.next_probe(want, m)
        expect_probe = -1 if worst >= m.sum() or m.sum() == 0 else p
        assert (ch.probe, ch.n_alive) == (expect_probe, int(m.sum()))
        if m.sum():
            assert (ch.worst, ch.n_classes) == (worst, n)


@pytest.mark.parametrize("target", [0, 7, 13, 22])
def test_adaptive_loop_matches_oracle(target):
    """Choose on the GPU, observe the target by replaying it on the chosen
    probe, keep the zero class of a one-probe inference, repeat."""
    torch, capi = need_gpu()
    cands, pool = SMALL_CANDS, SMALL_POOL
    carr, parr = capi.models(cands), capi.probes(pool)
    alive = np.ones(len(cands), dtype=bool)
    used = []
    for _ in range(len(pool)):
        ch = capi.pchase_plan_next_probe(carr, parr, _bitmap(alive))
        if ch.probe < 0:
            break
        p = int(ch.probe)
        one = capi.probes([pool[p]])
        n, _ = capi.pchase_trace_len(one[0])
        bits = torch.zeros((n + 31) // 32 + 1, dtype=torch.int32, device="cuda")
        misses = torch.zeros(2, dtype=torch.int64, device="cuda")
        say(f"  target {target}: observe probe {p}")
        capi.cache_replay_probes(capi.models([cands[target]]), one, np.zeros(1, np.uint32), np.zeros(1, np.uint32),
                                 None, misses, bits, np.zeros(1, np.uint64))
        _, zero = capi.infer_cache_params(one, carr, bits=bits, bitoff=np.zeros(1, np.uint64),
                                          probe_select=capi.PROBES_ALL, want_zero=True)
        keep = np.array([(zero[c // 32] >> (c % 32)) & 1 for c in range(len(cands))], dtype=bool)
        alive &= keep
        used.append(p)
    surv, used_ref = P.adaptive(orc, cands, pool, cands[target])
    assert used == used_ref
    assert np.nonzero(alive)[0].tolist() == surv


def test_planner_full_grid_sampled():
    """The benchmark's configuration (438 candidates x the 768-probe feature
    grid): class rows of 24 seeded probes against the oracle, and the first
    choice (all candidates alive) against the oracle's choice over those
    rows' full pool recomputed only where it can win."""
    torch, capi = need_gpu()
    cands = [(int(c["C"]), int(c["b"]), int(c["a"]), int(c["policy"])) for c in W.candidate_grid()]
    grid = capi.pchase_mlp_grid()
    pool = [(grid[i].n_bytes, grid[i].s_bytes, grid[i].passes) for i in range(grid.n)]
    cls = torch.full((len(pool) * len(cands),), -1, dtype=torch.int32, device="cuda")
    say(f"pchase_plan_next_probe full grid: {len(cands)} x {len(pool)}")
    alive = np.ones(len(cands), dtype=bool)
    ch = capi.pchase_plan_next_probe(capi.models(cands), grid, _bitmap(alive), cls)
    got = cls.cpu().numpy().reshape(len(pool), len(cands))
    rng = np.random.default_rng(768)
    sample = sorted(set(rng.choice(len(pool), size=24, replace=False).tolist()) | {int(ch.probe)})
    want = P.classes(orc, cands, [pool[p] for p in sample])
    for i, p in enumerate(sample):
        assert np.array_equal(got[p], want[i]), pool[p]
    # the chosen probe's score is the oracle's score of that row, and no
    # sampled row scores better
    worst, n = P.score(want[sample.index(int(ch.probe))], alive)
    assert (ch.worst, ch.n_classes) == (worst, n)
    for i, p in enumerate(sample):
        w2, n2 = P.score(want[i], alive)
        assert (w2, -n2, p) >= (worst, -n, int(ch.probe))
