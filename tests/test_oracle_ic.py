"""Pins for the oracle's IC-model sketches (Section 3, structured permutation
ranks and sketches for an IC model, as l -> infinity).

* Structured permutation: every chunk of n positions holds every node exactly
  once, and a node's place in a chunk is uniform.
* Coins of the per-position instances: live at rate (thr + 1) / 2^32, the two
  halves of one output uncorrelated, thr = 2^32 - 1 always live.
* p = 1 (every instance is the graph): X_u is the k smallest positions of the
  nodes u reaches, read off the permutation directly (brute-force reach).
* No edges: X_u is u's own position in each chunk.
* The reached positions: every chunk holds every node once, so the number of
  positions t <= k n whose node u reaches has expectation k Inf(u); their
  total over u, averaged over seeds, matches k times the exact IC influence
  (every live-edge subset of a tiny graph enumerated, exact fractions).
* The estimator n (k - 1) / (T - 1): without edges T = (k - 1) n + U with U
  uniform on 1..n, so its mean over seeds has a closed form.
* Every node holds exactly k positions, all at most k n.
"""
from fractions import Fraction

import numpy as np
import pytest

from workloads import from_edges
from brute import exact_ic_influence, reach, thr_prob

U32 = 0xFFFFFFFF


def test_order_is_a_structured_permutation(oracle_lib):
    n, k = 37, 9
    at = oracle_lib.ic_order(5, n, k)
    assert at.size == n * k
    for c in range(k):
        assert sorted(at[c * n:(c + 1) * n].tolist()) == list(range(n))
    # a node's place within its chunk is uniform over 0..n-1 (over chunks and seeds)
    n, k = 50, 64
    places = []
    for seed in range(40):
        at = oracle_lib.ic_order(seed, n, k).reshape(k, n)
        places.extend(np.where(at == 7)[1].tolist())
    places = np.array(places, dtype=np.float64)
    mean, sd = (n - 1) / 2, np.sqrt((n * n - 1) / 12) / np.sqrt(places.size)
    assert abs(places.mean() - mean) < 5 * sd
    assert np.unique(oracle_lib.ic_order(1, n, 2)[:n]).size == n


def test_instance_coins(oracle_lib):
    n = 100
    for thr, p in ((U32 // 2, 0.5), (U32 // 20, 0.05), (U32 // 100, 0.01)):
        hits = sum(oracle_lib.ic_live(3, n, u, (u + 1) % n, t, thr)
                   for u in range(40) for t in range(1, 101))
        N = 4000
        assert abs(hits / N - (thr + 1) / 2 ** 32) < 5 * np.sqrt(p * (1 - p) / N)
    assert all(oracle_lib.ic_live(9, n, 1, 2, t, U32) for t in range(1, 200))
    # instances 2j+1 and 2j+2 read the two halves of one output: uncorrelated
    a = np.array([oracle_lib.ic_live(4, n, 3, 4, 2 * j + 1, U32 // 2) for j in range(3000)])
    b = np.array([oracle_lib.ic_live(4, n, 3, 4, 2 * j + 2, U32 // 2) for j in range(3000)])
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / np.sqrt(3000)


def test_deterministic_graph_reads_the_permutation(oracle_lib):
    rng = np.random.default_rng(2)
    n, k, seed = 30, 6, 17
    src = rng.integers(0, n, 60)
    dst = rng.integers(0, n, 60)
    keep = src != dst
    pairs = sorted(set(zip(src[keep].tolist(), dst[keep].tolist())))
    g = from_edges(n, [p[0] for p in pairs], [p[1] for p in pairs])  # p = 1
    pos, est, _ = oracle_lib.ic_sketches(g, k, seed)
    at = oracle_lib.ic_order(seed, n, k)
    place = {}
    for t, v in enumerate(at.tolist(), start=1):
        place.setdefault(v, []).append(t)
    adj = [[] for _ in range(n)]
    for u, v in pairs:
        adj[u].append(v)
    for u in range(n):
        want = sorted(t for v in reach(adj, [u]) for t in place[v])[:k]
        assert pos[u].tolist() == want
        assert est[u] == (n * (k - 1)) / (want[-1] - 1)


def test_no_edges_own_positions(oracle_lib):
    n, k = 12, 5
    g = from_edges(n, [], [])
    pos, est, visits = oracle_lib.ic_sketches(g, k, 8)
    at = oracle_lib.ic_order(8, n, k).reshape(k, n)
    for u in range(n):
        own = [c * n + int(np.where(at[c] == u)[0][0]) + 1 for c in range(k)]
        assert pos[u].tolist() == own
    assert visits == n * k


def test_reached_positions_have_the_exact_expectation(oracle_lib):
    # Every chunk holds every node once and each position has its own
    # instance, so by linearity E[#{t <= k n : u reaches v_t}] = k Inf(u): the
    # visits, summed over u, have expectation k * sum_u Inf(u), exactly.
    # 5 nodes, 6 edges of probability 1/2 or 1/4: 64 live-edge subsets.
    edges = [(0, 1, U32 // 2), (1, 2, U32 // 2), (0, 3, U32 // 4), (3, 2, U32 // 2),
             (2, 4, U32 // 4), (4, 0, U32 // 2)]
    n, k = 5, 8
    g = from_edges(n, [e[0] for e in edges], [e[1] for e in edges],
                   [e[2] for e in edges])
    exact = sum(exact_ic_influence(n, [(u, v, thr_prob(t)) for u, v, t in edges], [x])[0]
                for x in range(n))
    trials = 600
    v = np.zeros(trials)
    for seed in range(trials):
        pos, est, visits = oracle_lib.ic_sketches(g, k, 1000 + seed)
        assert np.all(pos <= k * n) and np.all(np.diff(pos.astype(np.int64), axis=1) > 0)
        v[seed] = visits / k
    assert abs(v.mean() - float(exact)) < 5 * v.std() / np.sqrt(trials)


def test_estimator_closed_form_without_edges(oracle_lib):
    # Without edges X_u is u's own positions and T = (k-1) n + U, where the n
    # nodes take the places U = 1..n of the last chunk: the mean over nodes of
    # n (k-1) / (T-1) has a closed form, for every seed (slightly below the
    # influence 1, since structured ranks are not i.i.d.).
    for n, k in ((6, 5), (40, 64), (1, 2)):
        g = from_edges(n, [], [])
        want = sum(Fraction(n * (k - 1), (k - 1) * n + U - 1) for U in range(1, n + 1)) / n
        for seed in (3, 77, 2 ** 63 + 5):
            est = oracle_lib.ic_sketches(g, k, seed)[1]
            assert est.mean() == pytest.approx(float(want), rel=1e-13)
        assert float(want) <= 1.0


# ------------------------------------------------------------ union queries

def _sets(groups):
    off = np.zeros(len(groups) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(s) for s in groups])
    nodes = np.array([v for s in groups for v in s], dtype=np.uint32)
    return off, nodes


def test_union_of_one_is_the_node_estimate(oracle_lib):
    rng = np.random.default_rng(21)
    n, k = 40, 9
    src, dst = rng.integers(0, n, 100), rng.integers(0, n, 100)
    keep = src != dst
    pairs = sorted(set(zip(src[keep].tolist(), dst[keep].tolist())))
    g = from_edges(n, [p[0] for p in pairs], [p[1] for p in pairs], U32 // 3)
    pos, est, _ = oracle_lib.ic_sketches(g, k, 4)
    off, nodes = _sets([[u] for u in range(n)] + [[u, u, u] for u in range(n)])
    bk, st = oracle_lib.ic_union_query(pos, n, k, off, nodes, 0)
    assert np.all(st == 0)
    assert np.array_equal(bk, np.concatenate([est, est]))  # same operands, same division
    ck, _ = oracle_lib.ic_union_query(pos, n, k, off, nodes, 1)
    want = np.array([(k - 1) * n / (pos[u, k - 1] - 1.0) for u in range(n)] * 2)
    assert np.allclose(ck, want, rtol=1e-13)


def test_union_on_a_deterministic_graph_reads_the_permutation(oracle_lib):
    # p = 1: the union's positions are those of the nodes the set reaches
    rng = np.random.default_rng(22)
    n, k, seed = 30, 6, 19
    src, dst = rng.integers(0, n, 45), rng.integers(0, n, 45)
    keep = src != dst
    pairs = sorted(set(zip(src[keep].tolist(), dst[keep].tolist())))
    g = from_edges(n, [p[0] for p in pairs], [p[1] for p in pairs])
    pos, _, _ = oracle_lib.ic_sketches(g, k, seed)
    at = oracle_lib.ic_order(seed, n, k)
    place = {}
    for t, v in enumerate(at.tolist(), start=1):
        place.setdefault(v, []).append(t)
    adj = [[] for _ in range(n)]
    for u, v in pairs:
        adj[u].append(v)
    groups = [rng.choice(n, size=int(rng.integers(1, 6)), replace=False).tolist()
              for _ in range(40)]
    off, nodes = _sets(groups)
    est, _ = oracle_lib.ic_union_query(pos, n, k, off, nodes, 0)
    for j, S in enumerate(groups):
        T = sorted(t for v in reach(adj, S) for t in place[v])[k - 1]
        assert est[j] == (n * (k - 1)) / (T - 1)


def test_cohen_kaplan_adds_up_over_disjoint_sketches(oracle_lib):
    # no edges: sketches are disjoint, so every value has one holder and the
    # Cohen-Kaplan union is the sum of the members' (k-1) n / (T_u - 1)
    n, k = 25, 7
    g = from_edges(n, [], [])
    pos, _, _ = oracle_lib.ic_sketches(g, k, 5)
    groups = [[0, 1], [2, 3, 4, 5], list(range(n)), [], [7, 7, 8], [3, n]]
    off, nodes = _sets(groups)
    ck, st = oracle_lib.ic_union_query(pos, n, k, off, nodes, 1)
    assert st.tolist() == [0, 0, 0, 0, 0, -1] and ck[3] == 0.0 and ck[5] == 0.0
    for j in (0, 1, 2, 4):
        members = sorted(set(groups[j]))
        want = sum((k - 1) * n / (pos[u, k - 1] - 1.0) for u in members)
        assert ck[j] == pytest.approx(want, rel=1e-12)


def test_cohen_kaplan_overlapping_sketches_by_hand(oracle_lib):
    # Eq. unionest with permutation ranks: a position z held outside the
    # holders' own thresholds weighs n / (T_max(z) - 1), T_max the largest
    # threshold position among the sketches that hold it.  Worked by hand:
    # A = [1, 3, 5 | 7], B = [1, 4, 9 | 12], n = 10, k = 4.
    n, k = 10, 4
    pos = np.array([[1, 3, 5, 7], [1, 4, 9, 12]], dtype=np.uint32)
    off = np.array([0, 2, 3], dtype=np.uint64)
    nodes = np.array([0, 1, 0], dtype=np.uint32)
    est, st = oracle_lib.ic_union_query(pos, n, k, off, nodes, estimator=1)
    assert (st == 0).all()
    # {A, B}: 1 -> 10/11 (B's threshold, the larger), 3 -> 10/6, 4 -> 10/11,
    # 5 -> 10/6, 9 -> 10/11 (the smaller threshold for 1 would give 10/6).
    assert est[0] == pytest.approx(3 * 10 / 11 + 2 * 10 / 6, rel=1e-15)
    assert est[1] == pytest.approx(3 * 10 / 6, rel=1e-15)


def test_cohen_kaplan_unbiased_on_nested_reach_sets(oracle_lib):
    # p = 1 path 0 -> ... -> 99: R_25 is inside R_0, and the influence of
    # {0, 25} is 100 in every instance.  Shared positions weigh by the larger
    # threshold; the smaller one (the threshold of node 0) over-counts them,
    # which puts the mean near 118, about 50 standard errors away.
    n, k = 100, 16
    g = from_edges(n, list(range(n - 1)), list(range(1, n)), U32)
    off = np.array([0, 2], dtype=np.uint64)
    nodes = np.array([0, 25], dtype=np.uint32)
    ck = []
    for s in range(300):
        pos, _, _ = oracle_lib.ic_sketches(g, k, 700 + s)
        ck.append(oracle_lib.ic_union_query(pos, n, k, off, nodes, estimator=1)[0][0])
    ck = np.array(ck)
    assert abs(ck.mean() - 100) < 5 * ck.std() / np.sqrt(len(ck))
