"""Seeded influence-query workloads.

The paper queries seed sets whose nodes are drawn uniformly at random
(Section 6.2).  Query sets are returned in a CSR-like layout:
offsets uint64[Q+1] and nodes uint32[offsets[Q]]; the nodes of one set are
distinct (uniform sampling without replacement, by a partial Fisher-Yates
shuffle of [0, n)).
"""
from __future__ import annotations

import numpy as np


def _sets_from_sizes(rng, n: int, sizes: np.ndarray, chunk: int = 1 << 14):
    sizes = np.asarray(sizes, dtype=np.int64)
    if sizes.size and (sizes.min() < 0 or sizes.max() > n):
        raise ValueError("set size out of range")
    Q = sizes.shape[0]
    offsets = np.zeros(Q + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    nodes = np.empty(int(offsets[-1]), dtype=np.uint32)
    base = np.arange(n, dtype=np.int32)
    for q0 in range(0, Q, chunk):
        q1 = min(Q, q0 + chunk)
        sz = sizes[q0:q1]
        smax = int(sz.max()) if sz.size else 0
        if smax == 0:
            continue
        perm = np.tile(base, (q1 - q0, 1))
        rows = np.arange(q1 - q0)
        for j in range(smax):
            act = rows[sz > j]
            # pick uniformly from positions [j, n) and swap into position j
            pick = j + rng.integers(0, n - j, size=act.shape[0])
            a = perm[act, j].copy()
            perm[act, j] = perm[act, pick]
            perm[act, pick] = a
        for r in range(q1 - q0):
            s = int(sz[r])
            o = int(offsets[q0 + r])
            nodes[o:o + s] = perm[r, :s]
    return offsets, nodes


def lognormal_query_sets(Q: int, n: int, seed: int, mu: float = 2.0, sigma: float = 1.0,
                         lo: int = 1, hi: int = 512):
    """|S| = clamp(floor(exp(mu + sigma*Z) + 0.5), lo, hi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal(Q)
    sizes = np.clip(np.floor(np.exp(mu + sigma * z) + 0.5), lo, min(hi, n)).astype(np.int64)
    return _sets_from_sizes(rng, n, sizes)


def uniform_query_sets(Q: int, n: int, seed: int, lo: int = 1, hi: int = 512):
    """|S| uniform in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(lo, min(hi, n) + 1, size=Q)
    return _sets_from_sizes(rng, n, sizes)


def poisson_arrivals(rate: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of an open-loop Poisson stream: seeded exponential gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    expect = int(rate * duration_s * 1.2) + 64
    t = np.cumsum(rng.exponential(1.0 / rate, size=expect))
    while t[-1] < duration_s:
        more = np.cumsum(rng.exponential(1.0 / rate, size=expect)) + t[-1]
        t = np.concatenate([t, more])
    return t[t < duration_s]


def neighbourhood_query_sets(row_ptr: np.ndarray, col: np.ndarray, n: int, Q: int, s: int,
                             seed: int, max_tries: int = 64):
    """Seed sets whose members sit close together (the paper's neighbourhood
    generator, Section 6.2): pick a start node with probability proportional
    to its out-degree, grow a breadth-first search along out-edges level by
    level until the levels so far hold at least s nodes, and draw the s
    members uniformly without replacement from them.  A start whose search
    dies out below s nodes is redrawn (up to max_tries times; then the
    members are drawn uniformly from all nodes).  Returns (offsets, nodes)."""
    rng = np.random.default_rng(seed)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    outdeg = np.diff(row_ptr).astype(np.float64)
    if s > n:
        raise ValueError("set size out of range")
    prob = outdeg / outdeg.sum() if outdeg.sum() > 0 else None
    offsets = np.arange(Q + 1, dtype=np.uint64) * np.uint64(s)
    nodes = np.empty(Q * s, dtype=np.uint32)
    seen = np.zeros(n, dtype=bool)
    for q in range(Q):
        members = None
        for _ in range(max_tries if prob is not None else 0):
            u = int(rng.choice(n, p=prob))
            tree = [np.array([u], dtype=np.int64)]
            seen[u] = True
            count, frontier = 1, tree[0]
            while count < s and frontier.size:
                starts, ends = row_ptr[frontier], row_ptr[frontier + 1]
                idx = np.concatenate([np.arange(a, b) for a, b in zip(starts, ends)]) \
                    if frontier.size else np.empty(0, dtype=np.int64)
                nxt = np.unique(col[idx])
                nxt = nxt[~seen[nxt]]
                seen[nxt] = True
                tree.append(nxt)
                count += nxt.size
                frontier = nxt
            allnodes = np.concatenate(tree)
            seen[allnodes] = False
            if count >= s:
                members = rng.choice(allnodes, size=s, replace=False)
                break
        if members is None:
            members = rng.choice(n, size=s, replace=False)
        nodes[q * s:(q + 1) * s] = members
    return offsets, nodes
