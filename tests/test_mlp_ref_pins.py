"""Pins of the learned-proposer reference (oracle/mlp_ref.py).

The network reference is pinned by central finite differences of its own
forward pass (the analytic backward cannot agree with them by accident),
closed forms (zero weights, Adam under a constant gradient) and known bf16
roundings; the numpy Philox by the published known-answer vectors and by the
C oracle's independent copy; the features by the exact Eq. 2 form and the
no-miss case; the labels by the policy equivalences on uniform-stride
cycles; the noise by a per-bit loop over the C oracle's Philox.
"""
import os

import numpy as np
import pytest

from oracle import mlp_ref as R

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    return rows


def test_numpy_philox_known_answers():
    for r in _kat():
        out = R.philox4x32_10(*[np.array([v]) for v in r[:4]], r[4], r[5])
        assert [int(o[0]) for o in out] == r[6:10]


def test_numpy_philox_matches_c_oracle(orc):
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2**32, size=(64, 4), dtype=np.uint64)
    key = (0x12345678, 0x9ABCDEF0)
    got = np.stack(R.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], *key), axis=1)
    for i in range(64):
        ref = orc.philox([int(v) for v in ctr[i]], list(key))
        assert [int(v) for v in got[i]] == [int(v) for v in ref]


def test_bf16_rounding_ties_to_even():
    e = 2.0 ** -8
    cases = {1.0: 1.0, 1 + e: 1.0, 1 + 3 * e: 1 + 4 * e, 1 + e + 2.0 ** -20: 1 + 2 * e,
             -(1 + 3 * e): -(1 + 4 * e), 3.0: 3.0, 0.0: 0.0, 2.0 ** -130: 2.0 ** -130}
    for x, want in cases.items():
        assert float(R.bf16_round(np.float32(x))) == want, x


# ------------------------------------------------------ network ------
def _net(rng, n_in, n_h, n_out, scale=0.5):
    return [rng.normal(0, scale, (n_h, n_in)), rng.normal(0, 0.1, n_h),
            rng.normal(0, scale, (n_h, n_h)), rng.normal(0, 0.1, n_h),
            rng.normal(0, scale, (n_out, n_h)), rng.normal(0, 0.1, n_out)]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(11)
    params = _net(rng, 7, 6, 5)
    X = rng.normal(0, 1, (4, 7))
    y = np.array([0, 3, 4, 3])
    _, (_, a1, _, a2, _) = R.forward(params, X)
    assert np.abs(a1).min() > 1e-3 and np.abs(a2).min() > 1e-3   # no ReLU kink within reach of h
    _, grads = R.loss_and_grads(params, X, y)
    h = 1e-6
    for li, (p, g) in enumerate(zip(params, grads)):
        flat, gflat = p.reshape(-1), g.reshape(-1)
        for j in range(flat.size):
            old = flat[j]
            flat[j] = old + h
            lp = R.loss_fn(R.forward(params, X)[0], y)
            flat[j] = old - h
            lm = R.loss_fn(R.forward(params, X)[0], y)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[j]) <= 1e-6 * max(1.0, abs(fd)), (li, j, fd, gflat[j])


def test_zero_weights_closed_form():
    from scipy.special import logsumexp, softmax
    rng = np.random.default_rng(3)
    params = [np.zeros((6, 7)), rng.normal(0, 1, 6), np.zeros((6, 6)), rng.normal(0, 1, 6),
              np.zeros((5, 6)), rng.normal(0, 1, 5)]
    X = rng.normal(0, 1, (3, 7))
    y = np.array([1, 4, 0])
    z, _ = R.forward(params, X)
    assert np.allclose(z, params[5][None, :], atol=0)
    b3 = params[5]
    loss, grads = R.loss_and_grads(params, X, y)
    assert abs(loss - np.mean(logsumexp(b3) - b3[y])) < 1e-12
    onehot = np.eye(5)[y]
    assert np.allclose(grads[5], (softmax(b3)[None, :] - onehot).mean(axis=0), atol=1e-14)
    assert not np.any(grads[0]) and not np.any(grads[1])   # nothing flows back through W3 = 0


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are g and g^2
    at every step, so each step moves by lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 2.0, -1.0, 0.5])
    p, m, v = [p0], [np.zeros(4)], [np.zeros(4)]
    lr = 1e-3
    for t in range(1, 6):
        p, m, v = R.adam_step(p, [g], m, v, t, lr)
        want = p0 - t * lr * g / (np.abs(g) + 1e-8)
        assert np.allclose(p[0], want, rtol=0, atol=1e-12)


# ----------------------------------------------------- features ------
def test_grid_shape():
    g = R.grid()
    assert len(g) == 768 and g[0] == (4096, 32, 2) and g[255] == (4096 + 512 * 255, 32, 2)
    assert g[256] == (4096, 64, 2) and g[767] == (134656, 128, 2)


def test_features_exact_eq2_and_no_miss(orc):
    """C = 8 KB, b = 32 B, a = 4, T = 64, LRU: every N <= C gives 0; at
    s = b, N = C + m b with m = 16 (grid point i = 9) the steady pass has
    m (a + 1) = 80 misses out of N / s = 272 accesses (Eq. 2, exact); at
    N = 12 KB (i = 16) every set holds 6 > a lines and every access misses."""
    x = R.features(orc, (8192, 32, 4, 0))
    for si in range(3):
        for i in range(R.N_SIZES):
            if 4096 + 512 * i <= 8192:
                assert x[256 * si + i] == 0.0
    assert x[9] == np.float32(80 / 272)
    assert x[16] == 1.0


def test_canonical_labels_follow_policy_equivalences(orc):
    rows = [(8192, 32, 1, 0), (8192, 32, 1, 1), (8192, 32, 1, 2),
            (8192, 32, 2, 0), (8192, 32, 2, 1), (8192, 32, 2, 2),
            (8192, 64, 4, 0), (8192, 64, 4, 1)]
    lab = R.canonical_labels(orc, rows)
    # a = 1: all policies agree; a = 2: PLRU is LRU; LRU = FIFO on uniform cycles with s | N
    assert lab.tolist() == [0, 0, 0, 3, 3, 3, 6, 6]


def test_noise_mask_per_bit(orc):
    i, p, L, seed, thr = (1 << 33) + 7, 5, 61, 0xDEADBEEF12345, 20000
    got = R.flip_bits(i, p, L, seed, thr)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for k in range(L):
        out = orc.philox([k // 8, p, i & 0xFFFFFFFF, 0x80000000 | (i >> 32)], key)
        w = k % 8
        u16 = (int(out[w // 2]) >> (16 * (w % 2))) & 0xFFFF
        assert got[k] == (u16 < thr)


def test_noiseless_sample_is_clean_features(orc):
    rows = [(8192, 32, 4, 0), (12288, 64, 2, 2)]
    labels = np.array([0, 1])
    for i in range(3):
        x, y, (mi, base, thr) = R.sample(orc, i, 99, rows, labels, 0)
        assert thr == 0 and y == mi and base % 4 == 0 and base < rows[mi][1]
        assert np.array_equal(x, R.features(orc, rows[mi], base))
