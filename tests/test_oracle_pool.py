"""The oracle spread over processes gives what one process gives: every
(m, n), the best and the zero class of an exhaustive search, and every
replay's counts and hit bits, on small seeded workloads (CPU only)."""
import numpy as np

import oracle as orc
from oracle import pool
from paper_1509_02308_amd import workloads as W


def _obs(target, prows):
    hits_all, off, cfs, pos = [], [], [], 0
    m = orc.make_model(*target[:4])
    for r in prows:
        pr = orc.make_probe(*r)
        L = orc.cycle_len(pr)
        h, _, _ = orc.replay(m, orc.trace(pr), count_from=L)
        hits_all.append(h)
        off.append(pos)
        cfs.append(L)
        pos += len(h)
    return np.concatenate(hits_all), np.array(off, np.uint64), np.array(cfs, np.uint64)


def test_pool_inference_equals_one_process():
    cands = W.candidate_grid(Cs=(4096, 8192), bs=(32, 64), As=(1, 2, 4), policies=(0, 1, 2))
    crows = [tuple(int(x) for x in c) for c in cands]
    prows = [(N, s, 2) for s in (32, 64) for N in range(2048, 16384 + 1, 256)]
    flat, off, cf = _obs(crows[7], prows)
    best, m, n = orc.infer([orc.make_model(*r[:4]) for r in crows], [orc.make_probe(*r) for r in prows],
                           flat, off, cf, probe_select=0)
    pm, pn, pbest, pzero = pool.infer_scores(crows, prows, flat, off, cf, probe_select=0, procs=3)
    assert np.array_equal(pm, m) and np.array_equal(pn, n)
    assert pbest == best and pzero.tolist() == orc.zero_class(m).tolist()
    assert 7 in pzero.tolist()


def test_exact_argmin_definition():
    # 1/3 < 2/5 < 1/2; ties to the lowest index; n = 0 skipped
    assert pool.exact_argmin([1, 2, 1, 2], [2, 5, 3, 6]) == 2
    assert pool.exact_argmin([0, 5, 0], [0, 7, 9]) == 2
    assert pool.exact_argmin([0, 0], [0, 0]) == -1


def test_pool_replay_equals_one_process():
    mrows, prows = W.large_batch(60, seed=17, len_hi=3000, c_hi=64 << 10)
    om = [(int(r["C"]), int(r["b"]), int(r["a"]), int(r["policy"]), 0, int(r["seed"])) for r in mrows]
    op = [(int(p["N"]), int(p["s"]), int(p["passes"]), int(p["j0"]), int(p["base"])) for p in prows]
    cf = [orc.cycle_len(orc.make_probe(*p)) for p in op]
    seen = []
    tot, bits = pool.replay_probe_pairs(om, op, cf, bits_of=[3, 41], procs=2, chunk=7,
                                        progress=lambda d, n: seen.append((d, n)))
    assert seen[-1] == (60, 60)
    for i in range(60):
        h, mt, ms = orc.replay(orc.make_model(om[i][0], om[i][1], om[i][2], om[i][3], seed=om[i][5]),
                               orc.trace(orc.make_probe(*op[i])), base=op[i][4], trace_id=i, count_from=cf[i])
        assert (tot[i, 0], tot[i, 1]) == (mt, ms), i
        if i in (3, 41):
            assert np.array_equal(bits[i], h)
