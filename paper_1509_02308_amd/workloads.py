"""Seeded synthetic workloads (descriptors only).

This module is shared by the tests, the benchmark and the CPU reference as
the single source of inputs.  It enumerates probe descriptors (N, s, passes,
j0, base) and cache-model descriptors (C, b, a, policy, seed); it contains no
replay, no trace arithmetic and no scoring.  Sizes follow the paper's sweeps:
N ramps a line at a time across the capacity (Section 4.2 steps 2-3,
Section 4.3 texture L1 ramp 12 KB -> 12.5 KB), strides run from an element to
a few lines (Section 4.1, Eqs. (1)-(2)).
"""
from __future__ import annotations

import numpy as np

LRU, FIFO, PLRU, RANDOM, WRANDOM = 0, 1, 2, 3, 4
POLICY_NAMES = {LRU: "LRU", FIFO: "FIFO", PLRU: "PLRU", RANDOM: "RANDOM", WRANDOM: "WRANDOM"}

MODEL_DT = np.dtype([("C", "<u8"), ("b", "<u8"), ("a", "<u8"), ("policy", "<u8"),
                     ("set_shift", "<u8"), ("seed", "<u8")])
PROBE_DT = np.dtype([("N", "<u8"), ("s", "<u8"), ("base", "<u8"), ("j0", "<u8"),
                     ("elem", "<u8"), ("passes", "<u8")])


def models(rows) -> np.ndarray:
    """rows: iterable of (C, b, a, policy[, set_shift[, seed]])."""
    out = np.zeros(len(rows), dtype=MODEL_DT)
    for i, r in enumerate(rows):
        r = tuple(r) + (0,) * (6 - len(r))
        out[i] = r
    return out


def probes(rows) -> np.ndarray:
    """rows: iterable of (N, s[, passes[, j0[, base]]]); elem is 4 bytes (int32)."""
    out = np.zeros(len(rows), dtype=PROBE_DT)
    for i, r in enumerate(rows):
        N, s = r[0], r[1]
        passes = r[2] if len(r) > 2 else 2
        j0 = r[3] if len(r) > 3 else 0
        base = r[4] if len(r) > 4 else 0
        out[i] = (N, s, base, j0, 4, passes)
    return out


# --------------------------------------------------------------------------
# One LRU model, a P-chase sweep around its capacity (4 KB, 32 B lines,
# 4 ways): N = 2 KB .. 8 KB in 32 B steps, s in {32, 64, 128} B, 2 passes.
# --------------------------------------------------------------------------
def plain_sweep():
    model = models([(4096, 32, 4, LRU)])
    rows = [(N, s, 2) for s in (32, 64, 128) for N in range(2048, 8192 + 1, 32)]
    return model, probes(rows)


# --------------------------------------------------------------------------
# Candidate grid for the exhaustive search: C in {8..64 KB, powers of two and
# 1.5x}, b in {32, 64, 128} B, a in {1..64}, policy in {LRU, FIFO, PLRU};
# kept only when a*b divides C.  Canonical order: C, b, a, policy ascending.
# --------------------------------------------------------------------------
GRID_C = (8192, 12288, 16384, 24576, 32768, 49152, 65536)
GRID_B = (32, 64, 128)
GRID_A = (1, 2, 4, 8, 16, 32, 64)
GRID_POLICIES = (LRU, FIFO, PLRU)


def candidate_grid(Cs=GRID_C, bs=GRID_B, As=GRID_A, policies=GRID_POLICIES) -> np.ndarray:
    rows = []
    for C in Cs:
        for b in bs:
            for a in As:
                if C % (a * b) != 0:
                    continue
                for pol in policies:
                    rows.append((C, b, a, pol))
    return models(rows)


def own_sweep_rows(C: int, b: int, passes: int = 2):
    """The probes a candidate (C, b) replays: N = C/2 .. 2C step b, s in {b/2, b, 2b}."""
    return [(N, s, passes) for s in (b // 2, b, 2 * b) for N in range(C // 2, 2 * C + 1, b)]


def sweep_union(cands: np.ndarray, passes: int = 2) -> np.ndarray:
    """Distinct probes over every candidate's own sweep, sorted by (s, N)."""
    seen = set()
    for C, b in {(int(c["C"]), int(c["b"])) for c in cands}:
        for N, s, p in own_sweep_rows(C, b, passes):
            seen.add((s, N))
    rows = [(N, s, passes) for (s, N) in sorted(seen)]
    return probes(rows)


def pick_target(n_cands: int, seed: int = 1509) -> int:
    """The synthetic observed cache: one candidate drawn uniformly."""
    return int(np.random.default_rng(seed).integers(n_cands))


def inference_sweep(seed: int = 1509, Cs=GRID_C, bs=GRID_B, As=GRID_A, policies=GRID_POLICIES):
    cands = candidate_grid(Cs, bs, As, policies)
    return cands, sweep_union(cands), pick_target(len(cands), seed)


# --------------------------------------------------------------------------
# Large batch: (model, trace) pairs of uneven length, log-uniform on
# [lo, hi] accesses, realised as uniform-stride P-chases (s divides N so one
# pass is N/s accesses), models C in {2^k, 1.5*2^k} up to 4 MB, a up to 128,
# all four policies (RANDOM keyed by a per-model seed).
# --------------------------------------------------------------------------
def large_batch(n_pairs: int, seed: int = 4711, len_lo: int = 1000, len_hi: int = 100_000,
                c_lo: int = 8192, c_hi: int = 4 << 20, a_max: int = 128):
    rng = np.random.default_rng(seed)
    caps = []
    c = c_lo
    while c <= c_hi:
        caps.append(c)
        if c + c // 2 <= c_hi:
            caps.append(c + c // 2)
        c *= 2
    ways = [a for a in (1, 2, 4, 8, 16, 32, 64, 128) if a <= a_max]
    valid = [(C, b, a) for C in caps for b in (32, 64, 128) for a in ways if C % (a * b) == 0]
    pick = rng.integers(len(valid), size=n_pairs)
    pol = rng.integers(4, size=n_pairs)
    seeds = rng.integers(0, 2**63, size=n_pairs, dtype=np.int64).astype(np.uint64)
    mrows = [(valid[i][0], valid[i][1], valid[i][2], int(p), 0, int(sd))
             for i, p, sd in zip(pick, pol, seeds)]
    lens = np.exp(rng.uniform(np.log(len_lo), np.log(len_hi), size=n_pairs))
    strides = 4 << rng.integers(7, size=n_pairs)          # 4 B .. 256 B
    passes = rng.integers(1, 5, size=n_pairs)
    prow = []
    for L, s, p in zip(lens, strides, passes):
        per_pass = max(1, int(round(L / p)))
        prow.append((int(per_pass * s), int(s), int(p)))
    return models(mrows), probes(prow)


# --------------------------------------------------------------------------
# Non-uniform-stride chases (Section 5.2, Fig. 13(b)): rows
# (N, [(s_bytes, count), ...], passes, j0, base).
# --------------------------------------------------------------------------
def section52_rows(s1: int = 32 << 20, s2: int = 1 << 20, lines: int = 65, revisits: int = 3,
                   in_line: int = 64, passes: int = 2):
    """The Section 5.2 construction, scaled by its parameters: `lines` far
    steps of s1 over an array of lines * s1 bytes (every access a new line
    and page), the same lines `revisits` more times, `lines` steps of s2
    (s2 < s1: nearby pages), then `in_line` one-element steps."""
    N = lines * s1
    return [(N, [(s1, lines), (s1, lines * revisits), (s2, lines), (4, in_line)], passes, 0, 0)]


def nonuniform_rows(n: int = 48, seed: int = 52, n_lo: int = 64, n_hi: int = 4 << 20, max_count: int = 3000):
    """Random non-uniform chases: N log-uniform on [n_lo, n_hi] bytes, 1-8
    segments whose strides mix one element, a few lines, a large fraction of
    N, zero and more than N, counts 1..max_count, 1-3 passes, random start
    and base offset."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n):
        N = 4 * max(1, int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))) // 4)
        segs = []
        for _ in range(int(rng.integers(1, 9))):
            kind = int(rng.integers(5))
            if kind == 0:
                s = 4
            elif kind == 1:
                s = 4 * int(rng.integers(1, 129))
            elif kind == 2:
                s = 4 * int(rng.integers(0, N // 4))
            elif kind == 3:
                s = 0
            else:
                s = 4 * int(rng.integers(N // 4, 4 * (N // 4) + 1))
            segs.append((s, int(rng.integers(1, max_count + 1))))
        rows.append((N, segs, int(rng.integers(1, 4)), int(rng.integers(0, N // 4)), 4 * int(rng.integers(0, 1024))))
    return rows


# --------------------------------------------------------------------------
# Generalised caches (descriptors): the organisations of Sections 4.3-4.5
# as synthetic targets, and seeded random ones for parity tests.
# --------------------------------------------------------------------------
def paper_general_targets():
    """Dicts (line, ways per set, policy, set_shift, table, weights, name):
    * texture L1 (Sec. 4.3): 12 KB, 4 sets x 96 ways of 32 B, set from
      address bits 7-8;
    * read-only cache with a non-bit-field mapping (Sec. 4.3): the same
      geometry, set = a seeded table over 128 B blocks;
    * L2 TLB (Sec. 4.4, Fig. 9): 2 MB entries, one set of 17 and six of 8,
      a 65-entry table giving the large set 17 residues and each small set
      8 (residues 0..6 on sets 0..6);
    * Fermi L1 (Sec. 4.5): 16 KB, 32 sets x 4 ways of 128 B, way 2 replaced
      with probability 1/2 (weights 1, 3, 1, 1)."""
    rng = np.random.default_rng(980)
    return [
        {"name": "texture_l1", "line": 32, "ways": [96] * 4, "policy": LRU, "set_shift": 7},
        {"name": "readonly_table", "line": 32, "ways": [96] * 4, "policy": LRU, "set_shift": 7,
         "table": [int(x) for x in rng.permutation(np.arange(64) % 4)]},
        {"name": "l2_tlb", "line": 2 << 20, "ways": [17] + [8] * 6, "policy": LRU,
         "table": [r % 7 for r in range(56)] + [0] * 9},
        {"name": "fermi_l1", "line": 128, "ways": [4] * 32, "policy": WRANDOM, "weights": [1, 3, 1, 1],
         "seed": 1509},
    ]


def random_general(n: int, seed: int = 7):
    """Seeded random generalised caches: 1-12 sets of 1..128 ways (powers of
    two for PLRU), lines 4..128 B, all five policies, half with a set
    table, some with a set_shift, weights 0..7 per way (first > 0)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        pol = i % 5
        T = int(rng.integers(1, 13))
        if pol == PLRU:
            ways = [int(2 ** rng.integers(0, 8)) for _ in range(T)]
        else:
            ways = [int(rng.integers(1, 129)) if rng.random() < 0.3 else int(rng.integers(1, 17)) for _ in range(T)]
        line = int(4 << rng.integers(0, 6))
        d = {"line": line, "ways": ways, "policy": pol, "seed": int(rng.integers(0, 2 ** 40))}
        if rng.random() < 0.5:
            d["table"] = [int(x) for x in rng.integers(0, T, size=int(rng.integers(1, 40)))]
        if rng.random() < 0.3:
            d["set_shift"] = int(np.log2(line)) + int(rng.integers(0, 3))
        if pol == WRANDOM:
            w = [int(x) for x in rng.integers(0, 8, size=max(ways))]
            w[0] += 1
            d["weights"] = w
        out.append(d)
    return out


# --------------------------------------------------------------------------
# Generalised-candidate search (Sections 4.3-4.5): around each paper-shaped
# target, a family of neighbours that differ in one structural choice (set
# mapping bits, ways per set, set table, replacement weights, policy), and
# the fine-grained probes that observe it.
# --------------------------------------------------------------------------
def general_family(target: dict, seed: int = 1509):
    """Candidate dicts around a paper_general_targets() entry, the target
    itself included (at a seeded position).  Returns (family, index)."""
    rng = np.random.default_rng(seed)
    name = target["name"]
    fam = []
    if name == "texture_l1":
        for sh in (5, 6, 7, 8, 9):
            for pol in (LRU, FIFO):
                for w in (88, 96, 104):
                    fam.append({"line": 32, "ways": [w] * 4, "policy": pol, "set_shift": sh})
                fam.append({"line": 32, "ways": [48] * 8, "policy": pol, "set_shift": sh})
    elif name == "readonly_table":
        tables = [list(target["table"])] + [[int(x) for x in rng.permutation(np.arange(64) % 4)] for _ in range(7)]
        for sh in (6, 7, 8):
            for t in tables:
                fam.append({"line": 32, "ways": [96] * 4, "policy": LRU, "set_shift": sh, "table": t})
    elif name == "l2_tlb":
        plain = [r % 7 for r in range(7)]
        for pol in (LRU, FIFO):
            for big in (15, 16, 17, 18, 19):
                for small in (7, 8, 9):
                    for t in (list(target["table"]), plain):
                        fam.append({"line": 2 << 20, "ways": [big] + [small] * 6, "policy": pol, "table": t})
    elif name == "fermi_l1":
        for wts in ([1, 3, 1, 1], [1, 1, 1, 1], [3, 1, 1, 1], [1, 1, 3, 1], [1, 1, 1, 3]):
            for sd in (1509, 1510):
                fam.append({"line": 128, "ways": [4] * 32, "policy": WRANDOM, "weights": wts, "seed": sd})
        for pol in (LRU, FIFO, PLRU):
            fam.append({"line": 128, "ways": [4] * 32, "policy": pol})
    else:
        raise ValueError(f"no family for {name}")
    key = {k: v for k, v in target.items() if k != "name"}
    fam = [d for d in fam if d != key]
    at = int(rng.integers(0, len(fam) + 1))
    fam.insert(at, key)
    return fam, at


def general_probe_rows(target: dict, n_per_stride: int = 48, passes: int = 2):
    """Fine-grained probes (N, s, passes) for a generalised target: strides of
    half a line, a line, two lines and the set-mapping unit, N ramping from
    half to twice the capacity in n_per_stride steps of a line multiple."""
    b = int(target["line"])
    C = b * int(sum(target["ways"]))
    unit = 1 << int(target["set_shift"]) if target.get("set_shift") else b
    strides = sorted({s for s in (b // 2, b, 2 * b, unit) if s >= 4})
    rows = []
    for s in strides:
        step = max(b, (3 * C // 2) // n_per_stride // b * b)
        for N in range(C // 2, 2 * C + 1, step):
            rows.append((N, s, passes))
    return rows
