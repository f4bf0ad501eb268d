"""Tiny brute-force references used to pin the oracle (pure Python, small inputs).

These are independent of the oracle's C code paths: they take the live-edge
coin and the rank function as given (both are pinned on their own in
``test_oracle_random.py``) and recompute reachability, sketches, greedy
selection and exact IC expectations from the plain definitions.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def edge_list(g):
    src, dst = g.edges()
    return [(int(u), int(v), int(t)) for u, v, t in zip(src, dst, g.thr)]


def live_adjacency(g, seed, ell, oracle):
    """adj[i][u] = list of heads of live out-edges of u in instance i."""
    E = edge_list(g)
    adj = [[[] for _ in range(g.n)] for _ in range(ell)]
    for i in range(ell):
        for u, v, t in E:
            if oracle.live(seed, g.n, u, v, i, t):
                adj[i][u].append(v)
    return adj


def reach(adj_i, S):
    seen = set(S)
    stack = list(seen)
    while stack:
        u = stack.pop()
        for v in adj_i[u]:
            if v not in seen:
                seen.add(v)
                stack.append(v)
    return seen


def sketches(g, seed, ell, k, oracle, adj=None):
    """X_u by the definition: k smallest ranks over the combined reach set."""
    adj = adj or live_adjacency(g, seed, ell, oracle)
    X, size, R = [], [], []
    for u in range(g.n):
        ranks = sorted(oracle.rank(seed, v, i) for i in range(ell) for v in reach(adj[i], [u]))
        R.append(len(ranks))
        X.append(ranks[:k])
        size.append(min(k, len(ranks)))
    return X, size, R


def greedy_exact(g, seed, ell, s, oracle, adj=None):
    """Exact greedy on the l instances (max marginal gain, smallest id on ties)."""
    adj = adj or live_adjacency(g, seed, ell, oracle)
    sets = [set((v, i) for i in range(ell) for v in reach(adj[i], [u])) for u in range(g.n)]
    covered = set()
    seeds, gains = [], []
    chosen = set()
    for _ in range(s):
        best, bestg = None, -1
        for u in range(g.n):
            if u in chosen:
                continue
            gsz = len(sets[u] - covered)
            if gsz > bestg:
                best, bestg = u, gsz
        chosen.add(best)
        seeds.append(best)
        gains.append(bestg)
        covered |= sets[best]
    return seeds, gains


def exact_ic_influence(n, edges, S):
    """E[|reach(S)|] and Var by enumerating every live-edge subset.

    ``edges`` = [(u, v, p)] with p a Fraction; returns (mean, var) as Fractions.
    """
    m = len(edges)
    mean = Fraction(0)
    sq = Fraction(0)
    for mask in itertools.product((0, 1), repeat=m):
        pr = Fraction(1)
        adj = [[] for _ in range(n)]
        for b, (u, v, p) in zip(mask, edges):
            if b:
                pr *= p
                adj[u].append(v)
            else:
                pr *= 1 - p
        r = len(reach(adj, S))
        mean += pr * r
        sq += pr * r * r
    return mean, sq - mean * mean


def thr_prob(thr: int) -> Fraction:
    """Probability encoded by a threshold: P[coin <= thr] = (thr + 1) / 2^32."""
    return Fraction(int(thr) + 1, 1 << 32)


def random_small_graph(rng, n, m, thr_choices):
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    idx = rng.choice(len(pairs), size=min(m, len(pairs)), replace=False)
    src = np.array([pairs[j][0] for j in idx], dtype=np.int64)
    dst = np.array([pairs[j][1] for j in idx], dtype=np.int64)
    thr = rng.choice(np.array(thr_choices, dtype=np.uint64), size=src.size).astype(np.uint32)
    return src, dst, thr


# ------------------------------------------------------ inverting ranks
# SplitMix64 is a bijection (Steele, Lea, Flood 2014): every step of its
# finaliser is invertible (xorshifts by undoing the shifted bits, products by
# the inverse of the odd multiplier mod 2^64), and the counter is recovered
# from seed + (c + 1) * golden.  This turns a rank found in a sketch back into
# its node-instance pair, so large outputs can be checked pair by pair.
_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15
_MUL1 = 0xBF58476D1CE4E5B9
_MUL2 = 0x94D049BB133111EB


def _unxorshift(x, s):
    y = x.copy()
    for t in range(1, 64 // s + 1):
        y = x ^ (y >> np.uint64(s))
    return y


def rank_to_pair(ranks, seed):
    """Pair id 64 v + i of each rank (uint64 array in, uint64 array out)."""
    x = np.asarray(ranks, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _unxorshift(x, 31)
        z = z * np.uint64(pow(_MUL2, -1, 1 << 64))
        z = _unxorshift(z, 27)
        z = z * np.uint64(pow(_MUL1, -1, 1 << 64))
        z = _unxorshift(z, 30)
        c1 = (z - np.uint64(seed & _M64)) * np.uint64(pow(_GOLDEN, -1, 1 << 64))
        return c1 - np.uint64(1)
