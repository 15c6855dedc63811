"""Brute-force, declarative restatements used to pin the C oracle.

TEST INFRASTRUCTURE ONLY.  Pure Python, deliberately different in form from
``oracle.c`` so that a slip in one does not repeat in the other:

* LRU is stated as a reuse-distance rule (Section 4.1, Assumption 3): an
  access hits iff its line was used before and fewer than ``a`` distinct
  lines of the same set were used since.
* FIFO keeps a queue of resident lines per set (the hit/miss outcome of
  FIFO does not depend on which way a line sits in).
* Tree-PLRU is an explicit tree of node objects with lines at the leaves.
* RANDOM lists the ways of a set and draws the victim from an independent
  pure-Python Philox4x32-10 (Salmon et al., SC'11).
* The trace is Listing 1 + Listing 2 run literally on an array; the
  non-uniform chase is Fig. 13(b)'s array set up and chased the same way.
"""
from __future__ import annotations

from collections import deque

MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 from its published round function (SC'11, Sec. 3)."""
    x = [c & MASK32 for c in ctr]
    k = [key[0] & MASK32, key[1] & MASK32]
    for r in range(10):
        if r:
            k = [(k[0] + 0x9E3779B9) & MASK32, (k[1] + 0xBB67AE85) & MASK32]
        p0 = 0xD2511F53 * x[0]
        p1 = 0xCD9E8D57 * x[2]
        x = [((p1 >> 32) ^ x[1] ^ k[0]) & MASK32, p1 & MASK32,
             ((p0 >> 32) ^ x[3] ^ k[1]) & MASK32, p0 & MASK32]
    return x


def listing_trace(n_elems: int, stride: int, steps: int, j0: int = 0):
    """Listing 1 (A[i] = (i+stride) % size) then Listing 2 (j = A[j])."""
    A = [(i + stride) % n_elems for i in range(n_elems)]
    j = j0
    out = []
    for _ in range(steps):
        out.append(j)
        j = A[j]
    return out


def pointer_array_chase(n_elems: int, segments, steps: int, j0: int = 0):
    """Fig. 13(b) literally: initialise an array so that the element reached
    at position k of a pass points to the element of position k+1 (position
    of access k = j0 + sum of the strides taken before it, modulo the size),
    the last one back to j0, then chase j = A[j].  Only for segment lists
    that visit each element at most once per pass (else no such array
    exists: returns None)."""
    strides = [st for st, cnt in segments for _ in range(cnt)]
    pos = [(j0 + sum(strides[:k])) % n_elems for k in range(len(strides))]
    if len(set(pos)) != len(pos):
        return None
    A = [None] * n_elems
    for k, x in enumerate(pos):
        A[x] = pos[k + 1] if k + 1 < len(pos) else j0
    j, out = j0, []
    for _ in range(steps):
        out.append(j)
        j = A[j]
    return out


def lines_and_sets(idx, b, T, base=0, elem=4, set_shift=0):
    out = []
    for j in idx:
        addr = base + elem * j
        line = addr // b
        unit = (addr >> set_shift) if set_shift else line
        out.append((line, unit % T))
    return out


def lru_hits(idx, b, a, T, base=0, elem=4, set_shift=0):
    """Reuse-distance statement of LRU."""
    ls = lines_and_sets(idx, b, T, base, elem, set_shift)
    hits = []
    for k, (line, s) in enumerate(ls):
        last = None
        for q in range(k - 1, -1, -1):
            if ls[q][0] == line:
                last = q
                break
        if last is None:
            hits.append(0)
            continue
        between = {ls[q][0] for q in range(last + 1, k) if ls[q][1] == s}
        hits.append(1 if len(between) < a else 0)
    return hits


def fifo_hits(idx, b, a, T, base=0, elem=4, set_shift=0):
    queues = {}
    hits = []
    for line, s in lines_and_sets(idx, b, T, base, elem, set_shift):
        q = queues.setdefault(s, deque())
        if line in q:
            hits.append(1)
            continue
        hits.append(0)
        if len(q) == a:
            q.popleft()
        q.append(line)
    return hits


class _Node:
    __slots__ = ("bit", "left", "right", "line", "way")

    def __init__(self):
        self.bit = 0
        self.left = self.right = None
        self.line = None
        self.way = None


def _build_tree(lo: int, hi: int) -> _Node:
    n = _Node()
    if hi - lo == 1:
        n.way = lo
        return n
    mid = (lo + hi) // 2
    n.left = _build_tree(lo, mid)
    n.right = _build_tree(mid, hi)
    return n


def _leaves(n: _Node):
    if n.way is not None:
        return [n]
    return _leaves(n.left) + _leaves(n.right)


def _touch(root: _Node, way: int, a: int):
    """Every node on the path to ``way`` points to the other child."""
    node, lo, hi = root, 0, a
    while node.way is None:
        mid = (lo + hi) // 2
        if way < mid:
            node.bit = 1
            node, hi = node.left, mid
        else:
            node.bit = 0
            node, lo = node.right, mid


def _victim(root: _Node) -> _Node:
    node = root
    while node.way is None:
        node = node.right if node.bit else node.left
    return node


def plru_hits(idx, b, a, T, base=0, elem=4, set_shift=0):
    trees = {}
    hits = []
    for line, s in lines_and_sets(idx, b, T, base, elem, set_shift):
        root = trees.get(s)
        if root is None:
            root = trees[s] = _build_tree(0, a)
        leaves = _leaves(root)
        found = [lf for lf in leaves if lf.line == line]
        if found:
            hits.append(1)
            _touch(root, found[0].way, a)
            continue
        hits.append(0)
        empty = [lf for lf in leaves if lf.line is None]
        leaf = empty[0] if empty else _victim(root)
        leaf.line = line
        _touch(root, leaf.way, a)
    return hits


def random_hits(idx, b, a, T, seed, trace_id=0, base=0, elem=4, set_shift=0):
    ways = {}
    hits = []
    key = (seed & MASK32, seed >> 32)
    for k, (line, s) in enumerate(lines_and_sets(idx, b, T, base, elem, set_shift)):
        w = ways.setdefault(s, [None] * a)
        if line in w:
            hits.append(1)
            continue
        hits.append(0)
        if None in w:
            w[w.index(None)] = line
        else:
            r = philox4x32_10((k & MASK32, k >> 32, trace_id & MASK32, trace_id >> 32), key)
            w[r[0] % a] = line
    return hits


def hits_for(policy: int, idx, b, a, T, seed=0, trace_id=0, base=0, elem=4, set_shift=0):
    if policy == 0:
        return lru_hits(idx, b, a, T, base, elem, set_shift)
    if policy == 1:
        return fifo_hits(idx, b, a, T, base, elem, set_shift)
    if policy == 2:
        return plru_hits(idx, b, a, T, base, elem, set_shift)
    return random_hits(idx, b, a, T, seed, trace_id, base, elem, set_shift)


def general_hits(policy: int, idx, b, ways, table=None, weights=None, seed=0, trace_id=0, base=0, elem=4,
                 set_shift=0):
    """Generalised cache restated per set: set t has ways[t] ways; the set of
    an access is table[unit mod len(table)] (or unit mod len(ways)); LRU by
    reuse distance, FIFO by queue, tree-PLRU by node objects, RANDOM and
    weighted random by a list of ways and the pure-Python Philox (the weighted
    victim is found by walking the weights: u mod S falls in the w-th
    interval of widths weights[0], weights[1], ...)."""
    T = len(ways)
    seq = []
    for j in idx:
        addr = base + elem * j
        line = addr // b
        unit = (addr >> set_shift) if set_shift else line
        seq.append((line, table[unit % len(table)] if table is not None else unit % T))
    hits = []
    state = {}
    key = (seed & MASK32, seed >> 32)
    for k, (line, s) in enumerate(seq):
        a = ways[s]
        if policy == 0:
            last = None
            for q in range(k - 1, -1, -1):
                if seq[q][0] == line:
                    last = q
                    break
            if last is None:
                hits.append(0)
            else:
                between = {seq[q][0] for q in range(last + 1, k) if seq[q][1] == s}
                hits.append(1 if len(between) < a else 0)
            continue
        if policy == 1:
            q = state.setdefault(s, deque())
            if line in q:
                hits.append(1)
                continue
            hits.append(0)
            if len(q) == a:
                q.popleft()
            q.append(line)
            continue
        if policy == 2:
            root = state.get(s)
            if root is None:
                root = state[s] = _build_tree(0, a)
            leaves = _leaves(root)
            found = [lf for lf in leaves if lf.line == line]
            if found:
                hits.append(1)
                _touch(root, found[0].way, a)
                continue
            hits.append(0)
            empty = [lf for lf in leaves if lf.line is None]
            leaf = empty[0] if empty else _victim(root)
            leaf.line = line
            _touch(root, leaf.way, a)
            continue
        w = state.setdefault(s, [None] * a)
        if line in w:
            hits.append(1)
            continue
        hits.append(0)
        if None in w:
            w[w.index(None)] = line
            continue
        u = philox4x32_10((k & MASK32, k >> 32, trace_id & MASK32, trace_id >> 32), key)[0]
        if policy == 3:
            w[u % a] = line
        else:
            r = u % sum(weights[:a])
            v = 0
            while r >= weights[v]:
                r -= weights[v]
                v += 1
            w[v] = line
    return hits
