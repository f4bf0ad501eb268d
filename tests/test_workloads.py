"""The synthetic inputs follow their stated recipes (host logic only).

Graphs: simple directed graphs as sorted CSR (no self-loops, no duplicate
edges), with the stated sizes and degree shapes; thresholds are the integer
encodings of the stated edge probabilities.  Query workloads: set sizes from
the stated laws, members distinct and in range; Poisson arrivals with the
stated rate.  Also the bench's algorithmic byte counts, written out from
their definitions.
"""
import numpy as np

from workloads.configs import make_config, make_graph
from workloads.graphs import (UINT32_MAX, chung_lu_graph, er_graph, rmat_graph,
                              trivalency_thresholds, uniform_thresholds, wc_thresholds)
from workloads.queries import (lognormal_query_sets, neighbourhood_query_sets, poisson_arrivals,
                               uniform_query_sets)


def _check_simple_csr(n, row_ptr, col):
    row_ptr = row_ptr.astype(np.int64)
    assert row_ptr[0] == 0 and np.all(np.diff(row_ptr) >= 0) and row_ptr[-1] == col.size
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    assert np.all(col < n)
    assert not np.any(src == col), "self-loop"
    key = src.astype(np.int64) * n + col.astype(np.int64)
    assert np.all(np.diff(key) > 0), "rows not strictly increasing (or duplicate edge)"
    return src


def test_er_graph_exact_size_and_simple():
    rp, col = er_graph(300, 5000, seed=7)
    _check_simple_csr(300, rp, col)
    assert col.size == 5000
    # same seed, same graph; another seed, another graph
    rp2, col2 = er_graph(300, 5000, seed=7)
    assert np.array_equal(rp, rp2) and np.array_equal(col, col2)
    assert not np.array_equal(col, er_graph(300, 5000, seed=8)[1])


def test_chung_lu_power_law_shape():
    n, m = 20000, 200000
    rp, col = chung_lu_graph(n, m, 2.1, seed=3)
    src = _check_simple_csr(n, rp, col)
    assert col.size == m
    outdeg = np.bincount(src, minlength=n)
    indeg = np.bincount(col, minlength=n)
    # heavy tails on both sides: the largest degree dwarfs the mean, and the
    # top 1% of nodes hold a large share of the edges
    for d in (outdeg, indeg):
        assert d.max() > 50 * d.mean()
        top = np.sort(d)[::-1][: n // 100].sum()
        assert top > 0.25 * m


def test_rmat_graph_small_scale():
    scale = 12
    rp, col = rmat_graph(scale, 1 << 16, (0.57, 0.19, 0.19, 0.05), seed=5, chunks=4, threads=2)
    n = 1 << scale
    _check_simple_csr(n, rp, col)
    assert 0 < col.size <= 1 << 16
    indeg = np.bincount(col, minlength=n)
    assert indeg.max() > 20 * indeg.mean()  # skewed (a = 0.57)


def test_thresholds_encode_the_probabilities():
    assert np.all(uniform_thresholds(5, 20) == 214748364)     # p = 0.05
    assert np.all(uniform_thresholds(5, 100) == 42949672)     # p = 0.01
    t = trivalency_thresholds(30000, seed=9)
    vals, counts = np.unique(t, return_counts=True)
    assert set(vals.tolist()) == {429496729, 42949672, 4294967}
    assert np.all(np.abs(counts / t.size - 1 / 3) < 0.02)
    # weighted cascade: 1 / indeg(head) for every edge
    rp, col = er_graph(200, 3000, seed=11)
    thr = wc_thresholds(rp, col, 200)
    indeg = np.bincount(col, minlength=200)
    assert np.array_equal(thr, (UINT32_MAX // indeg[col].astype(np.uint64)).astype(np.uint32))
    # every head's in-edges sum to probability ~1
    p = (thr.astype(np.float64) + 1) / 2.0 ** 32
    sums = np.bincount(col, weights=p, minlength=200)
    assert np.all(np.abs(sums[indeg > 0] - 1.0) < 1e-6)


def test_configs_materialise_as_stated():
    g = make_graph(make_config("tiny-ic"))
    assert (g.n, g.m) == (1000, 8000)
    assert np.all(g.thr == 214748364)
    s = make_graph(make_config("served-skim"))
    assert (s.n, s.m) == (1000, 8000) and np.all(s.thr == 42949672)


def _check_sets(off, nodes, n, Q):
    off = off.astype(np.int64)
    assert off[0] == 0 and off.size == Q + 1 and np.all(np.diff(off) >= 1)
    assert np.all(nodes < n)
    for j in range(0, Q, max(1, Q // 500)):  # members distinct within a set
        s = nodes[off[j]:off[j + 1]]
        assert np.unique(s).size == s.size
    return np.diff(off)


def test_lognormal_query_sets_follow_the_law():
    Q = 200000
    off, nodes = lognormal_query_sets(Q, 1000, seed=4)
    sizes = _check_sets(off, nodes, 1000, Q)
    assert sizes.min() >= 1 and sizes.max() <= 512
    # E[clamp(round(e^(2+Z)), 1, 512)] ~ 12.18; P(size 1) ~ 5.5%
    assert abs(sizes.mean() - 12.18) < 0.25
    assert abs(np.mean(sizes == 1) - 0.055) < 0.005


def test_uniform_query_sets_and_poisson_arrivals():
    Q = 5000
    off, nodes = uniform_query_sets(Q, 1000, seed=6)
    sizes = _check_sets(off, nodes, 1000, Q)
    assert sizes.min() >= 1 and sizes.max() <= 512
    assert abs(sizes.mean() - 256.5) < 6
    t = poisson_arrivals(50000.0, 2.0, seed=12)
    assert np.all(np.diff(t) > 0) and t[-1] < 2.0
    assert abs(t.size - 100000) < 4 * np.sqrt(100000)
    gaps = np.diff(t)
    assert abs(gaps.mean() * 50000.0 - 1.0) < 0.02
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.03  # exponential: cv = 1


def test_bench_algorithmic_bytes():
    import bench
    cnt = {"c_min": 1000, "n_exp": 100, "n_ins": 500, "w_live": 700}
    assert bench.algorithmic_bytes_search(cnt) == 8 * 1000 + 16 * 100
    assert bench.algorithmic_bytes_build(cnt, n=10, k=4) == 8 * 1000 + 16 * 100 + 8 * 40 + 8 * 10
    assert bench.visit_model_bytes(cnt) == 500 * 56 + 700 * 20
    # the discrepancy-tail tree: 5 rows pair up as 5 -> 3 -> 2 -> 1 (4 pairs),
    # each pair sum_{j=0..bins} (j + 1) multiply-adds
    assert bench.tail_convolution_flops(5, 3) == 2 * 4 * (1 + 2 + 3 + 4)
    assert bench.tail_convolution_flops(1, 100) == 0


def _bfs_depths(row_ptr, col, n, u):
    depth = np.full(n, -1)
    depth[u] = 0
    frontier = [u]
    d = 0
    while frontier:
        d += 1
        nxt = []
        for x in frontier:
            for v in col[row_ptr[x]:row_ptr[x + 1]]:
                if depth[v] < 0:
                    depth[v] = d
                    nxt.append(int(v))
        frontier = nxt
    return depth


def test_neighbourhood_query_sets_stay_within_the_smallest_ball():
    rp, col = er_graph(400, 2400, seed=13)
    rp = rp.astype(np.int64)
    depths = {u: _bfs_depths(rp, col, 400, u) for u in range(400) if rp[u + 1] > rp[u]}
    for s in (1, 5, 40):
        off, nodes = neighbourhood_query_sets(rp, col, 400, 30, s, seed=s)
        sizes = _check_sets(off, nodes, 400, 30)
        assert np.all(sizes == s)
        for q in range(30):
            S = nodes[off[q]:off[q + 1]].astype(np.int64)
            # some start u has all of S within the smallest depth whose ball holds >= s nodes
            ok = False
            for u, dep in depths.items():  # starts have out-edges (chosen by out-degree)
                if np.any(dep[S] < 0):
                    continue
                need = 0
                while np.sum((dep >= 0) & (dep <= need)) < s:
                    need += 1
                if dep[S].max() <= need:
                    ok = True
                    break
            assert ok, (s, q)
    # reproducible, and different from uniform sets: members cluster
    a = neighbourhood_query_sets(rp, col, 400, 5, 40, seed=3)
    b = neighbourhood_query_sets(rp, col, 400, 5, 40, seed=3)
    assert np.array_equal(a[1], b[1])


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: bench.py says so and exits before touching a device
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
    assert r.stdout == ""
