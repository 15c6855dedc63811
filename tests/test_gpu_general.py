"""GPU parity of the generalised caches (per-set ways, set tables, weighted
random replacement) through cache_replay_general, bit-exact against the
CPU oracle: seeded random models on random, uniform and non-uniform traces,
and the paper-shaped targets of Sections 4.3-4.5."""
import numpy as np
import pytest

import oracle as orc
from paper_1509_02308_amd import workloads as W
from tests.gpu_common import need_gpu, say, unpack_bits

pytestmark = pytest.mark.gpu


def _orc_general(d):
    return orc.General(d["line"], d["ways"], d["policy"], d.get("set_shift", 0), d.get("table"),
                       d.get("weights"), d.get("seed", 0))


def _traces(rng):
    tr = [rng.integers(0, int(rng.integers(50, 6000)), size=int(rng.integers(1, 2500))).astype(np.int32)
          for _ in range(10)]
    for N, s, passes in [(4096, 32, 3), (12288 + 512, 32, 2), (65536 + 128, 128, 2), (2048, 4, 2)]:
        tr.append(orc.trace(orc.make_probe(N, s, passes=passes)))
    for r in W.nonuniform_rows(n=4, seed=61, n_hi=1 << 20, max_count=600):
        tr.append(orc.trace_nu(r[0], r[1], passes=r[2], j0=r[3]))
    # long enough to be replayed as parts by set (state permitting)
    tr.append(rng.integers(0, 20000, size=300001).astype(np.int32))
    tr.append(orc.trace(orc.make_probe(24576 + 128, 32, passes=20)))
    return tr


def _run(torch, capi, models, traces, bases, mode):
    off = np.concatenate([[0], np.cumsum([len(t) for t in traces])]).astype(np.uint64)
    idx = torch.from_numpy(np.concatenate(traces + [np.zeros(1, np.int32)])).cuda()
    pairs = [(m, t) for m in range(len(models)) for t in range(len(traces))]
    pm = np.array([m for m, _ in pairs], dtype=np.uint32)
    pt = np.array([t for _, t in pairs], dtype=np.uint32)
    cf = np.array([len(traces[t]) // 3 for _, t in pairs], dtype=np.uint64)
    words = [(len(traces[t]) + 31) // 32 for _, t in pairs]
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    bits = torch.full((int(sum(words)) + 1,), 0x77, dtype=torch.int32, device="cuda")
    misses = torch.full((2 * len(pairs),), -1, dtype=torch.int64, device="cuda")
    say(f"cache_replay_general mode={mode}: {len(models)} models, {len(pairs)} pairs")
    capi.cache_replay_general(capi.general_models(models), idx, off, bases, pm, pt, cf, misses, bits, bitoff, mode)
    torch.cuda.synchronize()
    mis = misses.cpu().numpy().astype(np.uint64).reshape(-1, 2)
    b = bits.cpu().numpy().view(np.uint32)
    for i, (m, t) in enumerate(pairs):
        hits, mt, ms = orc.replay_general(_orc_general(models[m]), traces[t], base=bases[t], trace_id=t,
                                          count_from=int(cf[i]))
        assert (mis[i, 0], mis[i, 1]) == (mt, ms), (models[m], t)
        assert np.array_equal(unpack_bits(b[bitoff[i]:], len(traces[t])), hits), (models[m], t)


@pytest.mark.parametrize("mode", [0, 1])
def test_general_random_models_match_oracle(mode):
    torch, capi = need_gpu()
    rng = np.random.default_rng(100 + mode)
    models = W.random_general(30, seed=8 + mode)
    for d in models:
        assert _orc_general(d).ok(), d
    traces = _traces(rng)
    bases = [4 * int(rng.integers(0, 2048)) for _ in traces]
    _run(torch, capi, models, traces, bases, mode)


def test_paper_shaped_targets_match_oracle():
    torch, capi = need_gpu()
    rng = np.random.default_rng(44)
    models = [{k: v for k, v in d.items() if k != "name"} for d in W.paper_general_targets()]
    traces = _traces(rng)
    page = 2 << 20
    for n in (64, 65, 66, 70):                     # the L2 TLB staircase: chases at s = 2 MB
        traces.append(orc.trace(orc.make_probe(n * page, page, passes=3)))
    traces.append(orc.trace(orc.make_probe(5 * 128 * 32, 128 * 32, passes=400)))   # Fermi L1 one-line overflow
    bases = [0] * len(traces)
    _run(torch, capi, models, traces, bases, 0)


def test_general_equal_sets_match_standard_replay():
    """A generalised model with equal sets and no table is the standard
    model: both entry points give the same bits and counts."""
    torch, capi = need_gpu()
    rng = np.random.default_rng(12)
    rows = [(4096, 32, 4, p, 0, 77) for p in range(4)] + [(12288, 32, 96, 0, 7, 0), (65536, 64, 128, 2, 0, 0)]
    gen = [{"line": b, "ways": [a] * (C // (a * b)), "policy": p, "set_shift": sh, "seed": sd}
           for C, b, a, p, sh, sd in rows]
    traces = _traces(rng)
    off = np.concatenate([[0], np.cumsum([len(t) for t in traces])]).astype(np.uint64)
    idx = torch.from_numpy(np.concatenate(traces + [np.zeros(1, np.int32)])).cuda()
    pairs = [(m, t) for m in range(len(rows)) for t in range(len(traces))]
    pm = np.array([m for m, _ in pairs], dtype=np.uint32)
    pt = np.array([t for _, t in pairs], dtype=np.uint32)
    words = [(len(traces[t]) + 31) // 32 for _, t in pairs]
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    out = []
    for name in ("standard", "general"):
        bits = torch.zeros(int(sum(words)) + 1, dtype=torch.int32, device="cuda")
        misses = torch.zeros(2 * len(pairs), dtype=torch.int64, device="cuda")
        say(f"equal sets through the {name} entry point")
        if name == "standard":
            capi.cache_replay_batch(capi.models(rows), idx, off, None, pm, pt, None, misses, bits, bitoff)
        else:
            capi.cache_replay_general(capi.general_models(gen), idx, off, None, pm, pt, None, misses, bits, bitoff)
        torch.cuda.synchronize()
        out.append((bits.cpu().numpy(), misses.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


# ------------------------------------------------ generalised-candidate search --
def _observe(target, rows):
    """The target's hit bits per probe (oracle replay, trace id = probe
    index), packed at word offsets, plus the flat bytes the oracle scores."""
    g = _orc_general(target)
    hits, words, off, cf = [], [], [], []
    pos = 0
    for i, r in enumerate(rows):
        p = orc.make_probe(*r)
        h, _, _ = orc.replay_general(g, orc.trace(p), trace_id=i)
        hits.append(h)
        off.append(pos)
        pos += len(h)
        cf.append(orc.cycle_len(p))
        n = (len(h) + 31) // 32
        pad = np.zeros(n * 32, np.uint8)
        pad[:len(h)] = h
        words.append((pad.reshape(n, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(1).astype(np.uint32))
    bitoff = np.concatenate([[0], np.cumsum([len(w) for w in words])[:-1]]).astype(np.uint64)
    return (np.concatenate(hits), np.array(off, np.uint64), np.array(cf, np.uint64),
            np.concatenate(words + [np.zeros(1, np.uint32)]), bitoff)


def _zero_list(zero, n):
    return [i for i in range(n) if (int(zero[i // 32]) >> (i % 32)) & 1]


@pytest.mark.parametrize("name", ["texture_l1", "readonly_table", "l2_tlb", "fermi_l1"])
def test_general_search_recovers_paper_targets(name):
    """Sections 4.3-4.5: the search over each paper-shaped target's family
    gives the oracle's (m, n) for every candidate, its best and its zero
    class, and the target is in that class."""
    torch, capi = need_gpu()
    target = [t for t in W.paper_general_targets() if t["name"] == name][0]
    fam, at = W.general_family(target)
    rows = W.general_probe_rows(target)
    flat, off, cf, packed, bitoff = _observe(target, rows)
    best, m, n = orc.infer_general([_orc_general(d) for d in fam], [orc.make_probe(*r) for r in rows], flat, off, cf)
    mn = torch.zeros(2 * len(fam), dtype=torch.int64, device="cuda")
    say(f"generalised search {name}: {len(fam)} candidates x {len(rows)} probes")
    res, zero = capi.infer_cache_params_general(capi.probes(rows), capi.general_models(fam),
                                                bits=torch.from_numpy(packed.view(np.int32)).cuda(), bitoff=bitoff,
                                                mn=mn, want_zero=True)
    got = mn.cpu().numpy().astype(np.uint64).reshape(-1, 2)
    assert np.array_equal(got[:, 0], m) and np.array_equal(got[:, 1], n)
    zc = [int(i) for i in np.nonzero(m == 0)[0]]
    assert res.best == best and (res.best_m, res.best_n) == (int(m[best]), int(n[best]))
    assert _zero_list(zero, len(fam)) == zc and res.n_zero == len(zc)
    assert at in zc and len(zc) < len(fam)


def test_general_search_from_latencies_and_with_a_plan():
    """The same search fed with latencies (hits fast, misses slow, jittered;
    the widest gap classifies them) and run inside a caller-owned plan."""
    torch, capi = need_gpu()
    target = [t for t in W.paper_general_targets() if t["name"] == "fermi_l1"][0]
    fam, at = W.general_family(target)
    rows = W.general_probe_rows(target)[::3]
    flat, off, cf, packed, bitoff = _observe(target, rows)
    rng = np.random.default_rng(5)
    lat = np.where(flat == 1, 90 + rng.integers(0, 20, flat.size), 400 + rng.integers(0, 60, flat.size)).astype(np.uint32)
    lat_off = np.concatenate([off, [flat.size]]).astype(np.uint64)
    best, m, n = orc.infer_general([_orc_general(d) for d in fam], [orc.make_probe(*r) for r in rows], flat, off, cf)
    say(f"generalised search from latencies: {len(fam)} x {len(rows)}")
    res, zero = capi.infer_cache_params_general(capi.probes(rows), capi.general_models(fam),
                                                lat=torch.from_numpy(lat.view(np.int32)).cuda(), lat_off=lat_off,
                                                want_zero=True)
    assert 90 <= res.threshold_used < 400
    assert res.best == best and _zero_list(zero, len(fam)) == [int(i) for i in np.nonzero(m == 0)[0]]
    plan = capi.Plan(256 << 20)
    try:
        mn = torch.zeros(2 * len(fam), dtype=torch.int64, device="cuda")
        res2, zero2 = capi.infer_cache_params_general(capi.probes(rows), capi.general_models(fam),
                                                      bits=torch.from_numpy(packed.view(np.int32)).cuda(),
                                                      bitoff=bitoff, mn=mn, want_zero=True, plan=plan)
        got = mn.cpu().numpy().astype(np.uint64).reshape(-1, 2)
        assert np.array_equal(got[:, 0], m) and np.array_equal(got[:, 1], n)
        assert res2.best == best and np.array_equal(zero2, zero)
    finally:
        plan.close()


def test_general_many_pairs_with_long_traces_split_by_length():
    """A call of at least 65,536 pairs (the schedule then splits a pair by
    length only above 131,072 accesses) with a few traces above that length:
    every policy of the generalised engine, all totals and the long pairs'
    bitmaps (and a sample of the short ones) against the oracle."""
    torch, capi = need_gpu()
    rng = np.random.default_rng(4096)
    models = W.random_general(10, seed=77)
    short = [rng.integers(0, int(rng.integers(16, 4000)), size=int(rng.integers(8, 64))).astype(np.int32)
             for _ in range(6560)]
    long_ = [rng.integers(0, 30000, size=140000 + 1000 * i).astype(np.int32) for i in range(3)]
    long_.append(orc.trace(orc.make_probe(36864 + 64, 64, passes=250)))   # 144,250 accesses
    traces = short + long_
    assert len(models) * len(traces) >= 65536 and min(len(t) for t in long_) > 131072
    off = np.concatenate([[0], np.cumsum([len(t) for t in traces])]).astype(np.uint64)
    idx = torch.from_numpy(np.concatenate(traces + [np.zeros(1, np.int32)])).cuda()
    pm = np.repeat(np.arange(len(models), dtype=np.uint32), len(traces))
    pt = np.tile(np.arange(len(traces), dtype=np.uint32), len(models))
    cf = np.array([len(traces[t]) // 2 for t in pt], dtype=np.uint64)
    words = np.array([(len(traces[t]) + 31) // 32 for t in pt], dtype=np.uint64)
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    bits = torch.full((int(words.sum()) + 1,), 0x55, dtype=torch.int32, device="cuda")
    misses = torch.full((2 * len(pm),), -1, dtype=torch.int64, device="cuda")
    bases = [4 * int(rng.integers(0, 4096)) for _ in traces]
    say(f"cache_replay_general: {len(models)} models x {len(traces)} traces = {len(pm)} pairs")
    capi.cache_replay_general(capi.general_models(models), idx, off, bases, pm, pt, cf, misses, bits, bitoff, 0)
    torch.cuda.synchronize()
    mis = misses.cpu().numpy().astype(np.uint64).reshape(-1, 2)
    b = bits.cpu().numpy().view(np.uint32)
    oms = [_orc_general(d) for d in models]
    n_long = len(long_)
    for i in range(len(pm)):
        m, t = int(pm[i]), int(pt[i])
        hits, mt, ms = orc.replay_general(oms[m], traces[t], base=bases[t], trace_id=t, count_from=int(cf[i]))
        assert (mis[i, 0], mis[i, 1]) == (mt, ms), (models[m], t)
        if t >= len(traces) - n_long or i % 97 == 0:
            assert np.array_equal(unpack_bits(b[bitoff[i]:], len(traces[t])), hits), (models[m], t)
