"""GPU parity of the non-uniform-stride chase (Section 5.2, Fig. 13(b)):
trace generation and replay through cache_replay_batch, bit-exact against
the CPU oracle."""
import numpy as np
import pytest

import oracle as orc
from paper_1509_02308_amd import workloads as W
from tests.gpu_common import need_gpu, orc_model, say, unpack_bits
from tests.test_gpu_parity import MODELS

pytestmark = pytest.mark.gpu

FIG13B = (96, [(32, 1), (16, 1), (8, 1), (16, 1), (8, 2), (80, 1), (8, 3)], 2, 0, 0)


def _rows():
    return [FIG13B] + W.section52_rows() + W.nonuniform_rows()


def _oracle_trace(r):
    return orc.trace_nu(r[0], r[1], passes=r[2], j0=r[3], base=r[4])


def _gpu_traces(torch, capi, rows):
    parr, sarr = capi.nu_probes(rows)
    total = sum(capi.pchase_trace_nu_len(parr, sarr, i)[0] for i in range(len(rows)))
    idx = torch.full((total + 7,), -1, dtype=torch.int32, device="cuda")
    off = capi.pchase_trace_nu(parr, sarr, idx)
    torch.cuda.synchronize()
    return idx, off


def test_nonuniform_trace_matches_oracle():
    torch, capi = need_gpu()
    rows = _rows()
    say(f"pchase_trace_nu: {len(rows)} probes")
    idx, off = _gpu_traces(torch, capi, rows)
    got = idx.cpu().numpy()
    assert (got[int(off[-1]):] == -1).all()                    # nothing written past the end
    for i, r in enumerate(rows):
        want = _oracle_trace(r)
        assert int(off[i + 1] - off[i]) == len(want)
        assert np.array_equal(got[int(off[i]):int(off[i + 1])], want), i


def test_nonuniform_long_trace_matches_oracle():
    """Millions of accesses per probe: many blocks, segment changes inside
    a thread's run and a ragged tail."""
    torch, capi = need_gpu()
    rows = [(1 << 30, [(4, 3_000_001), (4096 + 4, 999_999), (3 << 28, 7)], 2, 12345, 64),
            ((1 << 20) + 12, [(4 * 257, 2_500_003)], 3, 5, 0)]
    say("pchase_trace_nu: long traces")
    idx, off = _gpu_traces(torch, capi, rows)
    got = idx.cpu().numpy()
    for i, r in enumerate(rows):
        assert np.array_equal(got[int(off[i]):int(off[i + 1])], _oracle_trace(r)), i


@pytest.mark.parametrize("mode", [0, 1])
def test_nonuniform_replay_matches_oracle(mode):
    """Replay of the non-uniform traces on every way class and policy."""
    torch, capi = need_gpu()
    rows = [FIG13B] + W.section52_rows(s1=1 << 20, s2=1 << 14) + W.nonuniform_rows(n=16, seed=53, max_count=800)
    idx, off = _gpu_traces(torch, capi, rows)
    traces = [_oracle_trace(r) for r in rows]
    bases = [r[4] for r in rows]
    pairs = [(m, t) for m in range(len(MODELS)) for t in range(len(rows))]
    pm = np.array([m for m, _ in pairs], dtype=np.uint32)
    pt = np.array([t for _, t in pairs], dtype=np.uint32)
    cf = np.array([len(traces[t]) // 2 for _, t in pairs], dtype=np.uint64)
    words = [(len(traces[t]) + 31) // 32 for _, t in pairs]
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    bits = torch.full((int(sum(words)) + 1,), 0x55, dtype=torch.int32, device="cuda")
    misses = torch.full((2 * len(pairs),), -1, dtype=torch.int64, device="cuda")
    say(f"cache_replay_batch on non-uniform traces mode={mode}: {len(pairs)} pairs")
    capi.cache_replay_batch(capi.models(MODELS), idx, off, bases, pm, pt, cf, misses, bits, bitoff, mode)
    torch.cuda.synchronize()
    mis = misses.cpu().numpy().astype(np.uint64).reshape(-1, 2)
    b = bits.cpu().numpy().view(np.uint32)
    for i, (m, t) in enumerate(pairs):
        hits, mt, ms = orc.replay(orc_model(MODELS[m]), traces[t], base=bases[t], trace_id=t,
                                  count_from=int(cf[i]))
        assert (mis[i, 0], mis[i, 1]) == (mt, ms), (MODELS[m], t)
        assert np.array_equal(unpack_bits(b[bitoff[i]:], len(traces[t])), hits), (MODELS[m], t)


def test_nonuniform_lru_fifo_differ_on_gpu():
    """A revisit into a resident line separates LRU from FIFO; the GPU
    replay shows the same difference as the oracle."""
    torch, capi = need_gpu()
    n = 64
    rows = [(4 * n, [(32, 1), (4 * (n - 7), 1), (60, 1), (4 * (n - 14), 1), (4, 1)], 1, 0, 0)]
    idx, off = _gpu_traces(torch, capi, rows)
    mrows = [(64, 32, 2, W.LRU), (64, 32, 2, W.FIFO)]
    misses = torch.zeros(4, dtype=torch.int64, device="cuda")
    bits = torch.zeros(2, dtype=torch.int32, device="cuda")
    capi.cache_replay_batch(capi.models(mrows), idx, off, None, np.array([0, 1], np.uint32),
                            np.array([0, 0], np.uint32), None, misses, bits, np.array([0, 1], np.uint64))
    torch.cuda.synchronize()
    b = bits.cpu().numpy().view(np.uint32)
    assert unpack_bits(b[0:1], 5).tolist() == [0, 0, 1, 0, 1]
    assert unpack_bits(b[1:2], 5).tolist() == [0, 0, 1, 0, 0]


def test_nonuniform_benchmark_size_sampled():
    """The benchmark's non-uniform workload (4096 chases, 1.1e9 accesses):
    16 seeded traces compared whole with the oracle, and their replays
    through a standard and a generalised cache."""
    torch, capi = need_gpu()
    rows = W.nonuniform_rows(n=4096, seed=5209, n_hi=64 << 20, max_count=60_000)
    say("pchase_trace_nu at benchmark size")
    idx, off = _gpu_traces(torch, capi, rows)
    rng = np.random.default_rng(4096)
    sample = sorted(rng.choice(len(rows), size=16, replace=False).tolist())
    traces = []
    for i in sample:
        want = _oracle_trace(rows[i])
        got = idx[int(off[i]):int(off[i + 1])].cpu().numpy()
        assert np.array_equal(got, want), i
        traces.append(want)
    sub = torch.from_numpy(np.concatenate(traces + [np.zeros(1, np.int32)])).cuda()
    soff = np.concatenate([[0], np.cumsum([len(t) for t in traces])]).astype(np.uint64)
    bases = [rows[i][4] for i in sample]
    n = len(traces)
    misses = torch.zeros(2 * n, dtype=torch.int64, device="cuda")
    say("replay of the sampled traces")
    capi.cache_replay_batch(capi.models([(16384, 64, 8, W.PLRU)]), sub, soff, bases, np.zeros(n, np.uint32),
                            np.arange(n, dtype=np.uint32), None, misses)
    g = [d for d in W.paper_general_targets() if d["name"] == "fermi_l1"][0]
    gm = torch.zeros(2 * n, dtype=torch.int64, device="cuda")
    capi.cache_replay_general(capi.general_models([{k: v for k, v in g.items() if k != "name"}]), sub, soff, bases,
                              np.zeros(n, np.uint32), np.arange(n, dtype=np.uint32), None, gm)
    torch.cuda.synchronize()
    mis, gmis = misses.cpu().numpy().reshape(-1, 2), gm.cpu().numpy().reshape(-1, 2)
    og = orc.General(g["line"], g["ways"], g["policy"], weights=g["weights"], seed=g["seed"])
    for t in range(n):
        _, mt, ms = orc.replay(orc.make_model(16384, 64, 8, W.PLRU), traces[t], base=bases[t], trace_id=t)
        assert (mis[t, 0], mis[t, 1]) == (mt, ms)
        _, mt, ms = orc.replay_general(og, traces[t], base=bases[t], trace_id=t)
        assert (gmis[t, 0], gmis[t, 1]) == (mt, ms)
