"""Large-batch replay of materialised traces (cache_replay_batch): pairs of
uneven length (1e3..1e5 accesses, log-uniform), caches from 8 KB to 4 MB
with up to 128 ways and all four policies (RANDOM keyed per model, counter
= (access index, trace id)).  Every pair's miss totals and a 1% sample of
the per-access bitmaps must equal the CPU oracle's, in both schedules, at a
small batch and at the benchmark's full size."""
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


@pytest.mark.timeout(900)
def test_large_batch_full_size():
    """The benchmark's large batch at full size (1e6 pairs, 2.15e10 accesses,
    one call in the batched schedule): every pair's (misses_total,
    misses_steady) against the oracle (replayed in host processes), and a
    seeded 1% of the pairs' bitmaps."""
    from oracle import pool

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
    bw = bits.cpu().numpy().view(np.uint32)
    del bits
    sample = sorted(int(i) for i in np.random.default_rng(4711).choice(n, n // 100, replace=False))
    say(f"large batch full size: replayed; oracle on all pairs ({pool.default_procs()} processes)")
    om = [(int(r["C"]), int(r["b"]), int(r["a"]), int(r["policy"]), int(r["set_shift"]), int(r["seed"]))
          for r in mrows]
    op = [(int(p["N"]), int(p["s"]), int(p["passes"]), int(p["j0"]), int(p["base"])) for p in prows]
    last = [0]

    def progress(done, total):
        if done - last[0] >= total // 10 or done == total:
            last[0] = done
            say(f"large batch full size: oracle {done}/{total} pairs")

    want, hits = pool.replay_probe_pairs(om, op, cyc, bits_of=sample, progress=progress)
    bad = np.nonzero((mis != want).any(axis=1))[0]
    assert len(bad) == 0, (len(bad), [(int(i), om[int(i)], tuple(mis[i]), tuple(want[i])) for i in bad[:5]])
    say(f"large batch full size: all {n} totals equal; checking {len(sample)} bitmaps")
    for i in sample:
        got = unpack_bits(bw[int(bitoff[i]):int(bitoff[i]) + int(words[i])], int(lens[i]))
        assert np.array_equal(got, hits[i]), (i, om[i])
