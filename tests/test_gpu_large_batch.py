"""Large-batch replay of materialised traces (cache_replay_batch): pairs of
uneven length (1e3..1e5 accesses, log-uniform), caches from 8 KB to 4 MB
with up to 128 ways and all four policies (RANDOM keyed per model, counter
= (access index, trace id)).  Every pair's miss totals and a 1% sample of
the per-access bitmaps must equal the CPU oracle's, in both schedules (pairs above 8192 accesses are split
by set into parts that merge their outputs)."""
import numpy as np
import pytest

import oracle as orc
from paper_1509_02308_amd import workloads as W
from tests.gpu_common import need_gpu, orc_model, say, unpack_bits

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1])
def test_large_batch_shape_matches_oracle(mode):
    torch, capi = need_gpu()
    n = 1500
    mrows, prows = W.large_batch(n, seed=4711 + mode)
    marr, parr = capi.models(mrows), capi.probes(prows)
    lens, cyc = zip(*[capi.pchase_trace_len(parr[i]) for i in range(n)])
    lens, cyc = np.array(lens, np.uint64), np.array(cyc, np.uint64)
    total = int(lens.sum())
    say(f"large batch mode={mode}: {n} pairs, {total} accesses")
    idx = torch.zeros(total + 1, dtype=torch.int32, device="cuda")
    off = capi.pchase_trace(parr, idx)
    words = (lens + 31) // 32
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    bits = torch.zeros(int(words.sum()) + 1, dtype=torch.int32, device="cuda")
    misses = torch.full((2 * n,), -1, dtype=torch.int64, device="cuda")
    bases = np.array([int(p["base"]) for p in prows], np.uint64)
    pm = np.arange(n, dtype=np.uint32)
    capi.cache_replay_batch(marr, idx, off, bases, pm, pm, cyc, misses, bits, bitoff, mode)
    torch.cuda.synchronize()
    mis = misses.cpu().numpy().astype(np.uint64).reshape(-1, 2)
    b = bits.cpu().numpy().view(np.uint32)
    sample = set(np.random.default_rng(99).choice(n, n // 100, replace=False).tolist())
    sample |= set(np.argsort(-lens.astype(np.int64))[:10].tolist())   # the longest pairs are split by set
    for i in range(n):
        r = mrows[i]
        om = orc_model((int(r["C"]), int(r["b"]), int(r["a"]), int(r["policy"]), int(r["set_shift"]), int(r["seed"])))
        p = prows[i]
        tr = orc.trace(orc.make_probe(int(p["N"]), int(p["s"]), int(p["passes"]), int(p["j0"]), int(p["base"])))
        hits, mt, ms = orc.replay(om, tr, base=int(p["base"]), trace_id=i, count_from=int(cyc[i]))
        assert (mis[i, 0], mis[i, 1]) == (mt, ms), (i, tuple(r))
        if i in sample:
            assert np.array_equal(unpack_bits(b[int(bitoff[i]):], int(lens[i])), hits), (i, tuple(r))


def test_large_batch_full_size_sampled():
    """The benchmark's large batch at full size (1e6 pairs, 2.15e10 accesses,
    one call in the batched schedule): a seeded 1% of the pairs is checked
    against the oracle, bitmaps and both counts."""
    torch, capi = need_gpu()
    n = 1_000_000
    mrows, prows = W.large_batch(n)
    marr, parr = capi.models(mrows), capi.probes(prows)
    lc = np.array([capi.pchase_trace_len(parr[i]) for i in range(n)], dtype=np.uint64)
    lens, cyc = lc[:, 0], lc[:, 1]
    total = int(lens.sum())
    say(f"large batch full size: {n} pairs, {total} accesses")
    idx = torch.empty(total + 1, dtype=torch.int32, device="cuda")
    off = capi.pchase_trace(parr, idx)
    words = (lens + 31) // 32
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    bits = torch.zeros(int(words.sum()) + 1, dtype=torch.int32, device="cuda")
    misses = torch.full((2 * n,), -1, dtype=torch.int64, device="cuda")
    bases = np.array([int(p["base"]) for p in prows], np.uint64)
    pm = np.arange(n, dtype=np.uint32)
    capi.cache_replay_batch(marr, idx, off, bases, pm, pm, cyc, misses, bits, bitoff)
    torch.cuda.synchronize()
    del idx
    mis = misses.cpu().numpy().astype(np.uint64).reshape(-1, 2)
    sample = np.random.default_rng(4711).choice(n, n // 100, replace=False)
    bw = bits.cpu().numpy().view(np.uint32)
    say("large batch full size: replayed; checking the sample")
    for i in sample:
        i = int(i)
        r, p = mrows[i], prows[i]
        om = orc_model((int(r["C"]), int(r["b"]), int(r["a"]), int(r["policy"]), int(r["set_shift"]), int(r["seed"])))
        tr = orc.trace(orc.make_probe(int(p["N"]), int(p["s"]), int(p["passes"]), int(p["j0"]), int(p["base"])))
        hits, mt, ms = orc.replay(om, tr, base=int(p["base"]), trace_id=i, count_from=int(cyc[i]))
        assert (mis[i, 0], mis[i, 1]) == (mt, ms), (i, tuple(r))
        assert np.array_equal(unpack_bits(bw[int(bitoff[i]):int(bitoff[i]) + int(words[i])], int(lens[i])), hits), i
