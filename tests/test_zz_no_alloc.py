"""cache_replay_batch_static, the entry point that allocates nothing (its
descriptors live in the library's fixed per-GPU scratch array), called
through the C ABI: its counts and hit bits must equal cache_replay_batch's
on the same inputs, on two calls in a row, the second with a smaller input
(the scratch keeps the first call's contents), and a call whose descriptors
exceed the fixed scratch is rejected with PCHASE_ERANGE."""
import numpy as np
import pytest

from paper_1509_02308_amd import workloads as W
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu

ERANGE = -2


def _inputs(torch, capi, n, seed, len_hi, c_hi):
    mrows, prows = W.large_batch(n, seed=seed, len_hi=len_hi, c_hi=c_hi)
    marr, parr = capi.models(mrows), capi.probes(prows)
    lc = np.array([capi.pchase_trace_len(parr[i]) for i in range(n)], dtype=np.uint64)
    lens, cyc = lc[:, 0], lc[:, 1]
    idx = torch.empty(int(lens.sum()) + 1, dtype=torch.int32, device="cuda")
    off = capi.pchase_trace(parr, idx)
    words = (lens + 31) // 32
    bitoff = np.concatenate([[0], np.cumsum(words)[:-1]]).astype(np.uint64)
    bases = np.array([int(p["base"]) for p in prows], np.uint64)
    return marr, idx, off, bases, cyc, bitoff, int(words.sum()) + 1


def _both(torch, capi, inp, n):
    marr, idx, off, bases, cyc, bitoff, nw = inp
    pm = np.arange(n, dtype=np.uint32)
    out = []
    for fn in (capi.cache_replay_batch, capi.cache_replay_batch_static):
        misses = torch.full((2 * n,), -1, dtype=torch.int64, device="cuda")
        bits = torch.full((nw,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
        fn(marr, idx, off, bases, pm, pm, cyc, misses, bits, bitoff)
        torch.cuda.synchronize()
        out.append((misses.cpu().numpy(), bits.cpu().numpy()))
    return out


def test_static_replay_equals_allocating_replay_twice():
    torch, capi = need_gpu()
    # first call: caches up to 4 MB (pairs split by set merge into zeroed
    # outputs), all policies; second call: fewer, shorter pairs
    for n, seed, len_hi, c_hi in ((3000, 61, 30_000, 4 << 20), (700, 62, 5_000, 256 << 10)):
        say(f"no-alloc replay: {n} pairs (seed {seed})")
        inp = _inputs(torch, capi, n, seed, len_hi, c_hi)
        (m0, b0), (m1, b1) = _both(torch, capi, inp, n)
        assert (m0 >= 0).all()
        assert np.array_equal(m0, m1)
        assert np.array_equal(b0, b1)


def test_static_replay_rejects_oversized_calls():
    torch, capi = need_gpu()
    n = 1_300_000   # > 64 MiB of 56-byte work items
    marr = capi.models([(8192, 32, 4, 0)])
    probe = capi.probes([(4096, 4, 1)])
    idx = torch.empty(1025, dtype=torch.int32, device="cuda")
    off = capi.pchase_trace(probe, idx)
    pm = np.zeros(n, np.uint32)
    misses = torch.zeros(2 * n, dtype=torch.int64, device="cuda")
    say("no-alloc replay: oversized call")
    with pytest.raises(capi.PchaseError) as ei:
        capi.cache_replay_batch_static(marr, idx, off, None, pm, pm, None, misses)
    assert ei.value.code == ERANGE
