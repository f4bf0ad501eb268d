"""Pins for the oracle's union queries (Section 5.1).

* Bottom-k of the union: tau = k-th smallest distinct rank of the union of
  the sketches; estimate (k-1)/tau, or the exact count below k.  The union's
  bottom-k equals the bottom-k of the union of the reach sets, recomputed here
  by plain reachability; when the union holds fewer than k ranks the estimate
  is the exact influence.
* S = {u} reproduces the single-node estimate; the estimate is monotone in S.
* Set semantics: duplicates ignored, empty S gives 0, a bad node id flags
  only its own query.
* Cohen-Kaplan (eq. unionest): S = {u} and identical sketches reduce to the
  bottom-k estimate; unbiased over seeds.
"""
import numpy as np
import pytest

from workloads import from_edges
from brute import live_adjacency, reach, random_small_graph


def _qs(sets):
    off = np.zeros(len(sets) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(s) for s in sets])
    nodes = np.array([x for s in sets for x in s], dtype=np.uint32)
    return off, nodes


def test_single_node_matches_estimates(oracle_lib):
    rng = np.random.default_rng(1)
    src, dst, thr = random_small_graph(rng, 50, 150, [0xFFFFFFFF // 2, 0xFFFFFFFF // 10])
    g = from_edges(50, src, dst, thr)
    for ell, k in [(16, 8), (4, 64)]:
        ranks, size, _ = oracle_lib.build_alg2(g, 3, ell, k)
        est = oracle_lib.estimates(ranks, size, k, ell)
        off, nodes = _qs([[u] for u in range(50)])
        q, st = oracle_lib.union_query(ranks, size, k, ell, off, nodes)
        assert np.array_equal(q, est) and (st == 0).all()
        c, _ = oracle_lib.ck_query(ranks, size, k, ell, off, nodes)
        # one sketch: CK is (k-1)/tau as well, summed term by term (rounding only)
        assert np.allclose(c, est, rtol=1e-12, atol=0)


def test_union_is_bottom_k_of_union_of_reach_sets(oracle_lib):
    rng = np.random.default_rng(2)
    n, ell, k, seed = 40, 8, 10, 17
    src, dst, thr = random_small_graph(rng, n, 90, [0xFFFFFFFF // 3])
    g = from_edges(n, src, dst, thr)
    adj = live_adjacency(g, seed, ell, oracle_lib)
    ranks, size, _ = oracle_lib.build_alg2(g, seed, ell, k)
    sets = [list(rng.choice(n, size=int(rng.integers(1, 8)), replace=False)) for _ in range(60)]
    off, nodes = _qs(sets)
    est, _ = oracle_lib.union_query(ranks, size, k, ell, off, nodes)
    for S, e in zip(sets, est):
        U = sorted({oracle_lib.rank(seed, v, i) for i in range(ell) for v in reach(adj[i], S)})
        if len(U) < k:
            assert e == len(U) / ell
            assert e == oracle_lib.influence(g, seed, ell, S) / ell
        else:
            tau = U[k - 1]
            assert e == ((k - 1) / (((tau >> 11) + 1) * 2.0 ** -53)) / ell


def test_monotone_in_S(oracle_lib):
    rng = np.random.default_rng(3)
    n, ell, k = 60, 16, 16
    src, dst, thr = random_small_graph(rng, n, 200, [0xFFFFFFFF // 8])
    g = from_edges(n, src, dst, thr)
    ranks, size, _ = oracle_lib.build_alg2(g, 4, ell, k)
    for _ in range(20):
        perm = list(rng.permutation(n))
        sets = [perm[:j] for j in range(1, 25)]
        off, nodes = _qs(sets)
        est, _ = oracle_lib.union_query(ranks, size, k, ell, off, nodes)
        assert (np.diff(est) >= 0).all()


def test_set_semantics_and_status(oracle_lib):
    g = from_edges(10, [0, 1], [1, 2], 0xFFFFFFFF // 2)
    ranks, size, _ = oracle_lib.build_alg2(g, 1, 4, 4)
    off, nodes = _qs([[], [3, 3, 3], [3], [1, 99], [2, 0]])
    est, st = oracle_lib.union_query(ranks, size, 4, 4, off, nodes)
    assert est[0] == 0.0 and st[0] == 0
    assert est[1] == est[2]
    assert st[3] == -1 and est[3] == 0.0
    assert st[4] == 0
    c, cst = oracle_lib.ck_query(ranks, size, 4, 4, off, nodes)
    assert c[0] == 0.0 and c[1] == c[2] and cst[3] == -1


def test_ck_identical_sketches(oracle_lib):
    # 0 <-> 1 with p = 1: R_0 = R_1, identical full sketches; CK equals the
    # bottom-k union estimate, which equals the single-node estimate.
    g = from_edges(30, [0, 1] + [1] * 28, [1, 0] + list(range(2, 30)), 0xFFFFFFFF)
    ranks, size, _ = oracle_lib.build_alg2(g, 2, 8, 16)
    assert np.array_equal(ranks[0], ranks[1])
    off, nodes = _qs([[0, 1], [0]])
    c, _ = oracle_lib.ck_query(ranks, size, 16, 8, off, nodes)
    b, _ = oracle_lib.union_query(ranks, size, 16, 8, off, nodes)
    assert b[0] == b[1] and c[0] == c[1]
    assert np.allclose(c, b, rtol=1e-12, atol=0)


def test_ck_unbiased_on_disjoint_sets(oracle_lib):
    # two disjoint p=1 paths; Inf({0, 50}) = 100 exactly on every instance
    n, ell, k = 100, 8, 16
    src = list(range(49)) + list(range(50, 99))
    dst = list(range(1, 50)) + list(range(51, 100))
    g = from_edges(n, src, dst, 0xFFFFFFFF)
    off, nodes = _qs([[0, 50]])
    ck, bk = [], []
    for s in range(300):
        ranks, size, _ = oracle_lib.build_alg2(g, 900 + s, ell, k, threads=1)
        ck.append(oracle_lib.ck_query(ranks, size, k, ell, off, nodes)[0][0])
        bk.append(oracle_lib.union_query(ranks, size, k, ell, off, nodes)[0][0])
    ck, bk = np.array(ck), np.array(bk)
    assert abs(ck.mean() - 100) < 5 * ck.std() / np.sqrt(len(ck))
    assert abs(bk.mean() - 100) < 5 * bk.std() / np.sqrt(len(bk))
    assert ck.std() < bk.std()  # CK uses more of the sketches: lower variance


def _rank_for_rho(e):
    """A rank T whose real reading rho(T) = ((T >> 11) + 1) 2^-53 is exactly 2^-e."""
    return ((1 << (53 - e)) - 1) << 11


def test_ck_overlapping_sketches_by_hand(oracle_lib):
    # Eq. unionest: each distinct non-threshold value z of the union weighs
    # 1 / rho(max tau_u over the sketches holding z); a non-full holder has
    # tau = 1 (weight 1).  Values worked out by hand, with thresholds whose
    # real readings are exact powers of two (1/4 for A, 1/2 for B).
    k, ell = 4, 2
    ta, tb = _rank_for_rho(2), _rank_for_rho(1)
    z = 1 << 50  # held by A, B and C
    A = [z, 1 << 51, 1 << 52, ta]           # full, rho(tau) = 1/4
    B = [z, 1 << 53, 3 << 53, tb]           # full, rho(tau) = 1/2
    C = [z, 5 << 49]                        # not full: tau = 1
    NONE = 0xFFFFFFFFFFFFFFFF
    ranks = np.array([A, B, C + [NONE, NONE]], dtype=np.uint64)
    size = np.array([4, 4, 2], dtype=np.uint32)
    off, nodes = _qs([[0, 1], [0, 2], [0], [1, 2], [0, 1, 2]])
    c, st = oracle_lib.ck_query(ranks, size, k, ell, off, nodes)
    assert (st == 0).all()
    # {A, B}: z takes B's larger threshold (weight 2); A's other two values
    # weigh 4 each, B's other two 2 each: 2 + 4 + 4 + 2 + 2 = 14.  (Taking
    # the smaller threshold for z would give 16.)
    # {A, C}: z is held by the non-full C, weight 1: 1 + 4 + 4 + 1 = 10.
    # {A}: 3 values of weight 4 = 12 = (k - 1) / rho(tau).
    # {B, C}: 1 + 2 + 2 + 1 = 6.
    # {A, B, C}: 1 + 4 + 4 + 2 + 2 + 1 = 14.
    want = np.array([14.0, 10.0, 12.0, 6.0, 14.0]) / ell
    assert np.allclose(c, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("ell,k", [(1, 16), (8, 16)])
def test_ck_unbiased_on_nested_reach_sets(oracle_lib, ell, k):
    # A p = 1 path 0 -> 1 -> ... -> 99: R_25 is a subset of R_0 and
    # Inf({0, 25}) = 100 in every instance.  The ranks shared by the two
    # sketches must weigh 1 / rho of the LARGER threshold (tau_25 >= tau_0):
    # weighting them by the smaller one over-counts them, which puts the mean
    # near 118 (about 10 standard errors away over these seeds).
    n = 100
    g = from_edges(n, list(range(n - 1)), list(range(1, n)), 0xFFFFFFFF)
    off, nodes = _qs([[0, 25]])
    ck = []
    for s in range(300):
        ranks, size, _ = oracle_lib.build_alg2(g, 900 + s, ell, k, threads=1)
        ck.append(oracle_lib.ck_query(ranks, size, k, ell, off, nodes)[0][0])
    ck = np.array(ck)
    assert abs(ck.mean() - 100) < 5 * ck.std() / np.sqrt(len(ck))
