"""Reference for the learned candidate proposer: feature grid, training
samples, canonical labels and the fp64 3-layer MLP with Adam.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the test-suite,
the smoke check and the benchmark's CPU leg may use it; the HIP library
never does.  It shares no code with the HIP path.

What it computes
----------------
* Feature grid.  256 array sizes N_i = 4096 + 512 i bytes, i < 256, times
  strides s in {32, 64, 128} bytes, 2 passes each, start index 0.  These are
  the fine-grained runs of Section 4.2 (Fig. 6: N swept across the capacity,
  s around the line size), fixed once for every candidate.  Feature index
  = 256 * (stride slot) + i.  A feature is the steady-pass miss count of that
  probe divided by its cycle length L (the r of the average-latency model of
  Section 4.1), rounded once from the exact ratio to float32.
* Canonical label of a candidate.  The lowest-index candidate whose
  steady-pass hit/miss bits on the whole grid (base offset 0) equal its own:
  the representative of its zero class under "all probes".
* Training samples.  Sample i draws from Philox4x32-10 with key = seed and
  counter (i_lo, i_hi, 0, 0): the model (x mod n_models), a base offset
  4 * (y mod (b / 4)) and a flip threshold t = z mod (rho_q16 + 1).  The
  model is replayed on the grid at that base offset; steady-pass bit k of
  probe p is flipped when the 16-bit word (k mod 8) of
  Philox4x32-10(key = seed, counter = (k div 8, p, i_lo, 2^31 | i_hi)) is
  below t (word w is bits 16 (w mod 2) .. of output w div 2).  The feature
  is the noisy miss count / L; the label is the model's canonical label.
* Network.  h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3,
  loss = mean softmax cross-entropy, in float64 on given (bf16-representable)
  weights and inputs, with the analytic backward pass; Adam with
  beta = (0.9, 0.999), eps = 1e-8 and bias correction.
"""
from __future__ import annotations

import numpy as np

N_SIZES = 256
STRIDES = (32, 64, 128)
N_FEATURES = N_SIZES * len(STRIDES)
HIDDEN = 256


# ----------------------------------------------------------- grid ---
def grid():
    """(N, s, passes) of the 768 feature probes, in feature order."""
    return [(4096 + 512 * i, s, 2) for s in STRIDES for i in range(N_SIZES)]


# ------------------------------------------------------ philox (numpy) ---
def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 (Salmon et al., SC'11) on arrays of counters; returns
    the four output words as uint32 arrays."""
    M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
    W0, W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
    mask = np.uint64(0xFFFFFFFF)
    c = [np.asarray(v, dtype=np.uint64) & mask for v in (c0, c1, c2, c3)]
    c = np.broadcast_arrays(*c)
    c = [x.copy() for x in c]
    k0 = np.uint64(k0) & mask
    k1 = np.uint64(k1) & mask
    for _ in range(10):
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + W0) & mask
        k1 = (k1 + W1) & mask
    return [x.astype(np.uint32) for x in c]


# ----------------------------------------------------------- bf16 ---
def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16, ties to even, and
    return them as float32 (finite inputs)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32)


# ------------------------------------------------------- features ---
def _grid_replay(orc, model_row, base):
    """Steady-pass hit bits of every grid probe: list of uint8 arrays."""
    C, b, a, pol = model_row[:4]
    m = orc.make_model(C, b, a, pol)
    out = []
    for p, (N, s, passes) in enumerate(grid()):
        pr = orc.make_probe(N, s, passes, 0, base)
        L = orc.cycle_len(pr)
        hits, _, _ = orc.replay(m, orc.trace(pr), base=base, trace_id=p, count_from=L)
        out.append(np.asarray(hits[L:2 * L], dtype=np.uint8))
    return out


def ratio_f32(m, L) -> np.float32:
    """m / L rounded once to float32 (exact rational -> nearest float)."""
    return np.float32(np.float64(m) / np.float64(L))


def features(orc, model_row, base=0) -> np.ndarray:
    """768 clean features of one candidate (C, b, a, policy)."""
    steady = _grid_replay(orc, model_row, base)
    return np.array([ratio_f32(len(h) - int(h.sum()), len(h)) for h in steady], dtype=np.float32)


def canonical_labels(orc, model_rows) -> np.ndarray:
    """Lowest index with identical steady bits on the grid at base 0."""
    sig = [np.concatenate(_grid_replay(orc, r, 0)) for r in model_rows]
    lab = np.arange(len(model_rows), dtype=np.int32)
    for i in range(len(model_rows)):
        for j in range(i):
            if lab[j] == j and np.array_equal(sig[i], sig[j]):
                lab[i] = j
                break
    return lab


def sample_draw(i, seed, model_rows, rho_q16):
    """(model index, base offset, flip threshold) of sample i."""
    x = philox4x32_10(i & 0xFFFFFFFF, i >> 32, 0, 0, seed & 0xFFFFFFFF, seed >> 32)
    mi = int(x[0]) % len(model_rows)
    b = int(model_rows[mi][1])
    base = 4 * (int(x[1]) % (b // 4))
    thr = int(x[2]) % (rho_q16 + 1)
    return mi, base, thr


def flip_bits(i, p, L, seed, thr) -> np.ndarray:
    """uint8 flip mask of steady bits 0..L-1 of probe p in sample i."""
    k = np.arange(L, dtype=np.uint64)
    blk = k >> np.uint64(3)
    out = philox4x32_10(blk, p, i & 0xFFFFFFFF, 0x80000000 | (i >> 32), seed & 0xFFFFFFFF, seed >> 32)
    w = (k & np.uint64(7)).astype(np.int64)
    word = np.stack(out, axis=0)[w >> 1, np.arange(L)].astype(np.uint64)
    u16 = (word >> (np.uint64(16) * (w & 1).astype(np.uint64))) & np.uint64(0xFFFF)
    return (u16 < np.uint64(thr)).astype(np.uint8)


def sample(orc, i, seed, model_rows, labels, rho_q16):
    """Feature vector and label of training sample i."""
    mi, base, thr = sample_draw(i, seed, model_rows, rho_q16)
    steady = _grid_replay(orc, model_rows[mi], base)
    x = np.empty(N_FEATURES, dtype=np.float32)
    for p, h in enumerate(steady):
        L = len(h)
        noisy = h ^ flip_bits(i, p, L, seed, thr)
        x[p] = ratio_f32(L - int(noisy.sum()), L)
    return x, int(labels[mi]), (mi, base, thr)


# ------------------------------------------------------------ MLP ---
def forward(params, X):
    """params = (W1, b1, W2, b2, W3, b3) with W_l of shape (out, in); X of
    shape (batch, 768).  Returns (logits, cache) in float64."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return z, (X, a1, h1, a2, h2)


def loss_fn(z, y) -> float:
    """Mean softmax cross-entropy of logits z (batch, classes) at labels y."""
    zmax = z.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z - zmax).sum(axis=1)) + zmax[:, 0]
    return float(np.mean(lse - z[np.arange(len(y)), y]))


def loss_and_grads(params, X, y):
    """Loss and its gradient with respect to (W1, b1, W2, b2, W3, b3), by
    the chain rule through the softmax cross-entropy and both ReLUs."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    z, (X, a1, h1, a2, h2) = forward(params, X)
    B = z.shape[0]
    loss = loss_fn(z, y)
    zmax = z.max(axis=1, keepdims=True)
    e = np.exp(z - zmax)
    dz = e / e.sum(axis=1, keepdims=True)
    dz[np.arange(B), y] -= 1.0
    dz /= B
    gW3 = dz.T @ h2
    gb3 = dz.sum(axis=0)
    dh2 = (dz @ W3) * (a2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (a1 > 0)
    gW1 = dh1.T @ X
    gb1 = dh1.sum(axis=0)
    return loss, (gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (params, m, v)."""
    np_, nm, nv = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        p, g = np.asarray(p, np.float64), np.asarray(g, np.float64)
        mm = beta1 * np.asarray(mm, np.float64) + (1 - beta1) * g
        vv = beta2 * np.asarray(vv, np.float64) + (1 - beta2) * g * g
        mh = mm / (1 - beta1 ** t)
        vh = vv / (1 - beta2 ** t)
        np_.append(p - lr * mh / (np.sqrt(vh) + eps))
        nm.append(mm)
        nv.append(vv)
    return np_, nm, nv
