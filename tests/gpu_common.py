"""Helpers for the GPU parity tests: oracle-side expected values and the
packing of hit bytes into the library's bitmap layout.  Expected values come
from the CPU oracle only."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle as orc


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1509_02308_amd import capi
    capi.lib()
    return torch, capi


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def orc_model(row):
    C, b, a, pol = int(row[0]), int(row[1]), int(row[2]), int(row[3])
    sh = int(row[4]) if len(row) > 4 else 0
    seed = int(row[5]) if len(row) > 5 else 0
    return orc.make_model(C, b, a, pol, set_shift=sh, seed=seed)


def orc_probe(row):
    N, s = int(row[0]), int(row[1])
    passes = int(row[2]) if len(row) > 2 else 2
    j0 = int(row[3]) if len(row) > 3 else 0
    base = int(row[4]) if len(row) > 4 else 0
    return orc.make_probe(N, s, passes=passes, j0=j0, base=base)


def pack_bits(hits: np.ndarray) -> np.ndarray:
    """uint8 hit bytes -> uint32 words, bit k%32 of word k/32."""
    n = len(hits)
    words = (n + 31) // 32
    padded = np.zeros(words * 32, dtype=np.uint8)
    padded[:n] = hits
    bits = padded.reshape(words, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64)
    return bits.sum(axis=1).astype(np.uint32)


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    w = np.asarray(words, dtype=np.uint32).astype(np.uint64)
    b = ((w[:, None] >> np.arange(32, dtype=np.uint64)) & 1).astype(np.uint8).reshape(-1)
    return b[:n]
