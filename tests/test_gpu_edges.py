"""Edge cases on the GPU, each against the CPU oracle: empty calls, the
degenerate chases (one element, stride 0 or a multiple of N: L = 1; one
pass, so no steady access), the largest addresses the boundary accepts
(Ne just below 2^31, base offset just below 2^33), fully associative and
widest caches, a single candidate and an observation no candidate
reproduces."""
import numpy as np
import pytest

import oracle as orc
from paper_1509_02308_amd import workloads as W
from tests.gpu_common import need_gpu, orc_model, orc_probe, say, unpack_bits

pytestmark = pytest.mark.gpu

EDGE_PROBES = [
    (4, 4, 3), (4, 0, 2, 0, 12), (4096, 0, 2), (4096, 4096 * 3, 2),       # L = 1
    (4096, 32, 1),                                                        # one pass: nothing steady
    ((2 ** 31 - 2) * 4, (2 ** 30 - 1) * 4, 3, 5, 2 ** 33 - 4),            # Ne = 2^31 - 2, L = 2, top addresses
    ((2 ** 31 - 64) * 4, (2 ** 31 - 64) // 64 * 4, 3, 0, 2 ** 33 - 4096),  # L = 64 strides of 128 MB
    (13 * 4, 4, 4),
]
EDGE_MODELS = [
    (4096, 32, 128, W.LRU), (4096, 32, 128, W.FIFO), (4096, 32, 128, W.RANDOM, 0, 3),   # T = 1, widest
    (2048, 32, 64, W.PLRU),                                                             # T = 1, PLRU
    (4096, 4, 1, W.LRU), (1 << 30, 128, 128, W.LRU), (1 << 30, 128, 64, W.PLRU),        # direct-mapped; 1 GB
    (12288, 32, 96, W.LRU, 7),
]


def test_empty_calls_do_nothing():
    torch, capi = need_gpu()
    say("empty calls")
    off = capi.pchase_trace(capi.probes([]), None)
    assert off.tolist() == [0]
    misses = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    capi.cache_replay_probes(capi.models(EDGE_MODELS[:1]), capi.probes(EDGE_PROBES[:1]), np.zeros(0, np.uint32),
                             np.zeros(0, np.uint32), None, misses)
    capi.cache_replay_batch(capi.models(EDGE_MODELS[:1]), None, np.zeros(1, np.uint64), None, np.zeros(0, np.uint32),
                            np.zeros(0, np.uint32), None, misses)
    torch.cuda.synchronize()
    assert misses.cpu().tolist() == [-1, -1]


@pytest.mark.parametrize("mode", [0, 1])
def test_edge_probes_and_models_regenerated(mode):
    torch, capi = need_gpu()
    pairs = [(m, p) for m in range(len(EDGE_MODELS)) for p in range(len(EDGE_PROBES))]
    marr, parr = capi.models(EDGE_MODELS), capi.probes(EDGE_PROBES)
    lens = [orc.trace_len(orc_probe(EDGE_PROBES[p])) for _, p in pairs]
    words = [(n + 31) // 32 for n in lens]
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    bits = torch.full((int(sum(words)) + 1,), 0x11, dtype=torch.int32, device="cuda")
    misses = torch.full((2 * len(pairs),), -1, dtype=torch.int64, device="cuda")
    say(f"edge probes, regenerated traces, mode={mode}: {len(pairs)} pairs")
    capi.cache_replay_probes(marr, parr, np.array([m for m, _ in pairs], np.uint32),
                             np.array([p for _, p in pairs], np.uint32), None, misses, bits, bitoff, mode)
    torch.cuda.synchronize()
    mis = misses.cpu().numpy().astype(np.uint64).reshape(-1, 2)
    b = bits.cpu().numpy().view(np.uint32)
    for i, (m, p) in enumerate(pairs):
        op = orc_probe(EDGE_PROBES[p])
        hits, mt, ms = orc.replay(orc_model(EDGE_MODELS[m]), orc.trace(op), base=op.base, trace_id=p,
                                  count_from=orc.cycle_len(op))
        assert (mis[i, 0], mis[i, 1]) == (mt, ms), (EDGE_MODELS[m], EDGE_PROBES[p])
        assert np.array_equal(unpack_bits(b[bitoff[i]:], lens[i]), hits), (EDGE_MODELS[m], EDGE_PROBES[p])


def test_edge_probes_materialised():
    """The same chases materialised and replayed as traces, plus a trace of
    one access."""
    torch, capi = need_gpu()
    parr = capi.probes(EDGE_PROBES)
    total = sum(orc.trace_len(orc_probe(r)) for r in EDGE_PROBES)
    idx = torch.empty(total + 2, dtype=torch.int32, device="cuda")
    off = capi.pchase_trace(parr, idx)
    idx[total] = 9
    off = np.concatenate([off, [total + 1]]).astype(np.uint64)
    traces = [orc.trace(orc_probe(r)) for r in EDGE_PROBES] + [np.array([9], np.int32)]
    bases = [orc_probe(r).base for r in EDGE_PROBES] + [0]
    assert np.array_equal(idx[:total].cpu().numpy(), np.concatenate(traces[:-1]))
    pairs = [(m, t) for m in range(len(EDGE_MODELS)) for t in range(len(traces))]
    words = [(len(traces[t]) + 31) // 32 for _, t in pairs]
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    bits = torch.zeros(int(sum(words)) + 1, dtype=torch.int32, device="cuda")
    misses = torch.full((2 * len(pairs),), -1, dtype=torch.int64, device="cuda")
    say(f"edge probes materialised: {len(pairs)} pairs")
    capi.cache_replay_batch(capi.models(EDGE_MODELS), idx, off, bases, np.array([m for m, _ in pairs], np.uint32),
                            np.array([t for _, t in pairs], np.uint32), None, misses, bits, bitoff)
    torch.cuda.synchronize()
    mis = misses.cpu().numpy().astype(np.uint64).reshape(-1, 2)
    b = bits.cpu().numpy().view(np.uint32)
    for i, (m, t) in enumerate(pairs):
        hits, mt, ms = orc.replay(orc_model(EDGE_MODELS[m]), traces[t], base=bases[t], trace_id=t)
        assert (mis[i, 0], mis[i, 1]) == (mt, ms), (EDGE_MODELS[m], t)
        assert np.array_equal(unpack_bits(b[bitoff[i]:], len(traces[t])), hits), (EDGE_MODELS[m], t)


def test_inference_single_candidate_and_no_exact_match():
    """One candidate is its own best; when no candidate reproduces the
    observation, the best is the exact rational argmin of m / n."""
    torch, capi = need_gpu()
    prows = [(N, s, 2) for N in range(4096, 16385, 1024) for s in (32, 64)]
    parr = capi.probes(prows)
    lens = [orc.trace_len(orc_probe(r)) for r in prows]
    bitoff = np.concatenate([[0], np.cumsum([(n + 31) // 32 for n in lens])[:-1]]).astype(np.uint64)
    # observation: a cache outside the candidate list (3 ways, 6 KB, PLRU-free)
    target = (6144, 32, 3, W.FIFO)
    obs = np.zeros(int(bitoff[-1]) + (lens[-1] + 31) // 32 + 1, dtype=np.uint32)
    for p, r in enumerate(prows):
        op = orc_probe(r)
        h, _, _ = orc.replay(orc_model(target), orc.trace(op))
        padded = np.zeros(((len(h) + 31) // 32) * 32, np.uint64)
        padded[:len(h)] = h
        obs[int(bitoff[p]):int(bitoff[p]) + len(padded) // 32] = (padded.reshape(-1, 32) << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)
    bits = torch.from_numpy(obs.view(np.int32)).cuda()
    cands = [(4096, 32, 4, W.LRU), (8192, 32, 4, W.LRU), (8192, 64, 2, W.PLRU), (16384, 32, 8, W.FIFO)]
    for sel in (cands[:1], cands):
        say(f"inference with {len(sel)} candidate(s), no exact match")
        res, _ = capi.infer_cache_params(parr, capi.models(sel), bits=bits, bitoff=bitoff,
                                         probe_select=capi.PROBES_ALL)
        m, n = [], []
        ocands = [orc_model(c) for c in sel]
        flat = np.concatenate([unpack_bits(obs[int(bitoff[p]):], lens[p]) for p in range(len(prows))])
        offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
        cf = np.array([orc.cycle_len(orc_probe(r)) for r in prows], np.uint64)
        best, mm, nn = orc.infer(ocands, [orc_probe(r) for r in prows], flat, offs, cf, probe_select=0)
        assert res.best == best and (res.best_m, res.best_n) == (int(mm[best]), int(nn[best]))
        assert res.n_zero == 0 and res.best_m > 0
