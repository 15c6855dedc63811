"""pchase_abort: with the host flag set before a batched call, the call
returns PCHASE_EABORTED (an inference before it launches anything; a
materialised replay when its persistent kernels, which poll the flag on
their first queue pull, have drained), and once the flag is cleared the
very next call on the same inputs is exact against the oracle again."""
import numpy as np
import pytest

import oracle as orc
from paper_1509_02308_amd import workloads as W
from tests.gpu_common import need_gpu, orc_model, orc_probe, pack_bits, say

pytestmark = pytest.mark.gpu

EABORTED = -5


def _observation(crows, prows, target):
    om = orc_model(crows[target])
    hits, off, cfs, pos = [], [], [], 0
    for i, r in enumerate(prows):
        op = orc_probe(r)
        h, _, _ = orc.replay(om, orc.trace(op), base=op.base, trace_id=i)
        hits.append(h)
        off.append(pos)
        pos += len(h)
        cfs.append(orc.cycle_len(op))
    words = [(len(h) + 31) // 32 for h in hits]
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    packed = np.concatenate([pack_bits(h) for h in hits] + [np.zeros(1, np.uint32)])
    return hits, np.array(off, np.uint64), np.array(cfs, np.uint64), packed, bitoff


def test_abort_inference_then_exact():
    torch, capi = need_gpu()
    cands = W.candidate_grid(Cs=(4096, 8192, 16384), bs=(32, 64), As=(1, 2, 4, 8, 16), policies=(0, 1, 2))
    crows = [tuple(int(x) for x in c) for c in cands]
    prows = [(int(p["N"]), int(p["s"]), int(p["passes"])) for p in W.sweep_union(cands)]
    target = 11
    hits, off, cfs, packed, bitoff = _observation(crows, prows, target)
    bits = torch.from_numpy(packed.view(np.int32)).cuda()
    parr, carr = capi.probes(prows), capi.models(crows)
    say(f"abort: inference over {len(crows)} candidates, {len(prows)} probes, flag set")
    capi.pchase_abort(True)
    try:
        with pytest.raises(capi.PchaseError) as ei:
            capi.infer_cache_params(parr, carr, bits=bits, bitoff=bitoff, probe_select=1)
        assert ei.value.code == EABORTED
    finally:
        capi.pchase_abort(False)
    say("abort: flag cleared, same call again")
    mn = torch.zeros(2 * len(crows), dtype=torch.int64, device="cuda")
    res, _ = capi.infer_cache_params(parr, carr, bits=bits, bitoff=bitoff, probe_select=1, mn=mn)
    best, m, n = orc.infer([orc_model(r) for r in crows], [orc_probe(r) for r in prows],
                           np.concatenate(hits), off, cfs, probe_select=1)
    got = mn.cpu().numpy().astype(np.uint64).reshape(-1, 2)
    assert np.array_equal(got[:, 0], m) and np.array_equal(got[:, 1], n)
    assert res.best == best and m[target] == 0


def test_abort_materialised_replay_then_exact():
    torch, capi = need_gpu()
    n = 400
    mrows, prows = W.large_batch(n, seed=31, len_hi=20_000, c_hi=1 << 20)
    marr, parr = capi.models(mrows), capi.probes(prows)
    lc = np.array([capi.pchase_trace_len(parr[i]) for i in range(n)], dtype=np.uint64)
    lens, cyc = lc[:, 0], lc[:, 1]
    idx = torch.empty(int(lens.sum()) + 1, dtype=torch.int32, device="cuda")
    off = capi.pchase_trace(parr, idx)
    misses = torch.full((2 * n,), -1, dtype=torch.int64, device="cuda")
    bases = np.array([int(p["base"]) for p in prows], np.uint64)
    pm = np.arange(n, dtype=np.uint32)
    say(f"abort: materialised replay of {n} pairs, flag set")
    capi.pchase_abort(True)
    try:
        with pytest.raises(capi.PchaseError) as ei:
            capi.cache_replay_batch(marr, idx, off, bases, pm, pm, cyc, misses)
        assert ei.value.code == EABORTED
    finally:
        capi.pchase_abort(False)
    say("abort: flag cleared, same call again")
    capi.cache_replay_batch(marr, idx, off, bases, pm, pm, cyc, misses)
    torch.cuda.synchronize()
    mis = misses.cpu().numpy().astype(np.uint64).reshape(-1, 2)
    for i in range(n):
        r, p = mrows[i], prows[i]
        om = orc_model((int(r["C"]), int(r["b"]), int(r["a"]), int(r["policy"]), int(r["set_shift"]), int(r["seed"])))
        tr = orc.trace(orc.make_probe(int(p["N"]), int(p["s"]), int(p["passes"]), int(p["j0"]), int(p["base"])))
        _, mt, ms = orc.replay(om, tr, base=int(p["base"]), trace_id=i, count_from=int(cyc[i]))
        assert (mis[i, 0], mis[i, 1]) == (mt, ms), (i, tuple(r))
