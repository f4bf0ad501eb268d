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
