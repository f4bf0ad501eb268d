"""Pins for the oracle's combined reachability sketches and estimates.

* Definition (Section 3, eq. combinedrs): X_u = k smallest ranks over
  R_u = {(v, i) : u reaches v in G^(i)}; recomputed here in Python by plain
  per-instance reachability.
* Algorithm 2 (Section 5.2) must reproduce the definition exactly.
* Special cases: l = 1 (single-instance reachability sketches), p = 1
  (bottom-k of reach(u) x [l]), no edges (own ranks), k > |R_u| (all of R_u).
* Estimator (Section 3, eq. combinedthresh): |X_u| when |X_u| < k, which then
  equals the exact influence l * Inf({u}) / l; otherwise unbiased with
  CV at most 1/sqrt(k-2), checked over many seeds.
* Work counters of Algorithm 2 against direct sums over (v, i).
"""
import numpy as np
import pytest

from workloads import from_edges
from workloads.configs import make_config, make_graph
from brute import live_adjacency, reach, random_small_graph, sketches

UMAX = np.uint64(0xFFFFFFFFFFFFFFFF)


def _padded(X, k):
    out = np.full((len(X), k), UMAX, dtype=np.uint64)
    for u, row in enumerate(X):
        out[u, :len(row)] = row
    return out


@pytest.mark.parametrize("ell,k", [(1, 2), (1, 16), (2, 3), (16, 4), (16, 16), (64, 64), (5, 7)])
def test_alg2_equals_definition(oracle_lib, ell, k):
    rng = np.random.default_rng(ell * 100 + k)
    for trial in range(4):
        n = int(rng.integers(2, 30))
        m = int(rng.integers(0, 3 * n))
        src, dst, thr = random_small_graph(rng, n, m, [0xFFFFFFFF, 0xFFFFFFFF // 2,
                                                       0xFFFFFFFF // 4, 0xFFFFFFFF // 20])
        g = from_edges(n, src, dst, thr)
        seed = int(rng.integers(0, 2 ** 63))
        X, size, R = sketches(g, seed, ell, k, oracle_lib)
        ranks, sz, cnt = oracle_lib.build_alg2(g, seed, ell, k, threads=3)
        assert np.array_equal(ranks, _padded(X, k))
        assert np.array_equal(sz, np.array(size, dtype=np.uint32))
        rb, sb, reach_b = oracle_lib.sketch_brute(g, seed, ell, k)
        assert np.array_equal(rb, ranks) and np.array_equal(sb, sz)
        assert np.array_equal(reach_b, np.array(R, dtype=np.uint64))


def test_deterministic_graph_special_case(oracle_lib):
    rng = np.random.default_rng(3)
    n, ell, k = 25, 8, 12
    src, dst, _ = random_small_graph(rng, n, 40, [0xFFFFFFFF])
    g = from_edges(n, src, dst, 0xFFFFFFFF)
    adj = [[] for _ in range(n)]
    for a, b in zip(src, dst):
        adj[int(a)].append(int(b))
    ranks, size, _ = oracle_lib.build_alg2(g, 5, ell, k)
    for u in range(n):
        want = sorted(oracle_lib.rank(5, v, i) for v in reach(adj, [u]) for i in range(ell))[:k]
        assert list(ranks[u, :len(want)]) == want and size[u] == len(want)


def test_no_edges_gives_own_ranks(oracle_lib):
    n, ell, k = 30, 16, 5
    g = from_edges(n, [], [])
    ranks, size, _ = oracle_lib.build_alg2(g, 8, ell, k)
    own = np.sort(oracle_lib.ranks(8, n, ell), axis=1)[:, :k]
    assert np.array_equal(ranks, own) and (size == k).all()


def test_k_above_reach_keeps_everything_and_estimate_is_exact(oracle_lib):
    rng = np.random.default_rng(4)
    n, ell, k = 40, 8, 200
    src, dst, thr = random_small_graph(rng, n, 60, [0xFFFFFFFF // 3])
    g = from_edges(n, src, dst, thr)
    ranks, size, _ = oracle_lib.build_alg2(g, 21, ell, k)
    est = oracle_lib.estimates(ranks, size, k, ell)
    for u in range(n):
        infl = oracle_lib.influence(g, 21, ell, [u])  # l * Inf({u}) = |R_u|
        assert size[u] == infl
        assert est[u] == infl / ell  # bit-exact: |X_u| / l
        assert (ranks[u, size[u]:] == UMAX).all()


def test_alg2_on_tiny_config_matches_definition(oracle_lib):
    cfg = make_config("tiny-ic")
    g = make_graph(cfg)
    ranks, size, _ = oracle_lib.build_alg2(g, cfg["seed"], cfg["ell"], cfg["k"])
    nodes = np.arange(0, g.n, 7, dtype=np.uint32)
    rb, sb, _ = oracle_lib.sketch_brute(g, cfg["seed"], cfg["ell"], cfg["k"], nodes)
    assert np.array_equal(ranks[nodes], rb) and np.array_equal(size[nodes], sb)


def test_counters_match_direct_sums(oracle_lib):
    rng = np.random.default_rng(9)
    n, ell, k = 30, 6, 4
    src, dst, thr = random_small_graph(rng, n, 70, [0xFFFFFFFF // 2, 0xFFFFFFFF])
    g = from_edges(n, src, dst, thr)
    seed = 77
    adj = live_adjacency(g, seed, ell, oracle_lib)
    indeg = g.in_degree()
    n_ins = w_live = n_exp = c_min = 0
    for v in range(n):
        Ev = []
        for i in range(ell):
            E = min(k, len(reach(adj[i], [v])))
            live_in = sum(1 for u in range(n) if v in adj[i][u])
            n_ins += E
            w_live += E * live_in
            Ev.append(E)
        n_exp += max(Ev)
        c_min += max(Ev) * int(indeg[v])
    _, _, cnt = oracle_lib.build_alg2(g, seed, ell, k)
    assert cnt == {"n_ins": n_ins, "w_live": w_live, "n_exp": n_exp, "c_min": c_min}


def test_table3_layout_is_n_k_8_bytes(oracle_lib):
    # Table 3's sketch space column is exactly n * k * 8 bytes (e.g. AstroPh
    # 14.8K nodes, k = 64: 7.2 MiB); the sketch table here has that layout.
    g = from_edges(10, [0], [1])
    ranks, size, _ = oracle_lib.build_alg2(g, 1, 4, 64)
    assert ranks.dtype == np.uint64 and ranks.nbytes == 10 * 64 * 8
    assert round(14_800 * 64 * 8 / 2 ** 20, 1) == 7.2


def test_estimator_unbiased_with_bounded_cv(oracle_lib):
    # p = 1 path of 100 nodes: |R_0| = 100 * l exactly; the bottom-k estimate
    # over independent seeds must be unbiased with CV <= 1/sqrt(k-2).
    n, ell, k = 100, 16, 16
    g = from_edges(n, list(range(n - 1)), list(range(1, n)), 0xFFFFFFFF)
    true = n  # Inf({0}) on every instance
    vals = []
    for s in range(400):
        ranks, size, _ = oracle_lib.build_alg2(g, 5000 + s, ell, k, threads=1)
        vals.append(oracle_lib.estimates(ranks[:1], size[:1], k, ell)[0])
    vals = np.array(vals)
    cv_bound = 1 / np.sqrt(k - 2)
    assert abs(vals.mean() - true) < 5 * cv_bound * true / np.sqrt(len(vals))
    assert vals.std() / true < cv_bound * 1.15


def test_budgeted_brute_force_matches_and_aborts(oracle_lib):
    """The budgeted, threaded form of the definition returns the same sketches
    as the plain one, and leaves out exactly the nodes whose searches would
    scan more out-edges than the budget."""
    from brute import random_small_graph
    from workloads import from_edges
    rng = np.random.default_rng(77)
    src, dst, thr = random_small_graph(rng, 120, 500, [0xFFFFFFFF, 0xFFFFFFFF // 3])
    g = from_edges(120, src, dst, thr)
    R0, S0, reach0 = oracle_lib.sketch_brute(g, 5, 8, 6)
    R1, S1, reach1, ok = oracle_lib.sketch_brute(g, 5, 8, 6, budget=1 << 40, threads=3)
    assert ok.all() and np.array_equal(R0, R1) and np.array_equal(S0, S1)
    assert np.array_equal(reach0, reach1)
    outdeg = np.diff(g.row_ptr.astype(np.int64))
    R2, S2, _, ok2 = oracle_lib.sketch_brute(g, 5, 8, 6, budget=0, threads=2)
    assert np.array_equal(ok2, outdeg == 0)  # zero budget: only nodes with nothing to scan
    assert np.array_equal(R2[ok2], R0[ok2]) and np.array_equal(S2[ok2], S0[ok2])
