"""GPU parity of the structured permutation ranks for finite l (Section 3.1):
skim_build_sketches_perm's sketches (positions), sizes and estimates equal
the oracle's (Algorithm 2 with the oracle's own positions) bit for bit, and
skim_perm_query_batch's bottom-k and Cohen-Kaplan unions equal the oracle's.
Cases: random small graphs over (l, k) (k below and above l), the tiny-ic and
served-skim graphs, a 20,000-node weighted-cascade Chung-Lu graph, p = 1 and
edgeless graphs, and every search level taken by pull."""
import numpy as np
import pytest

from workloads import from_edges, uniform_query_sets
from workloads.configs import make_config, make_graph
from brute import random_small_graph
from gpu_util import dev, log, to_dev_u32, to_dev_u64

pytestmark = pytest.mark.gpu

U32 = 0xFFFFFFFF


def _build(g, ell, k, seed):
    import torch
    import paper_1408_6282_amd as sk
    G = sk.DeviceGraph.from_host(g, dev())
    ranks = torch.empty(g.n * k, dtype=torch.int64, device=dev())
    size = torch.empty(g.n, dtype=torch.int32, device=dev())
    est = torch.empty(g.n, dtype=torch.float64, device=dev())
    sk.skim_build_sketches_perm(G, ell, k, seed, ranks, size, est)
    torch.cuda.synchronize()
    return (ranks.cpu().numpy().view(np.uint64).reshape(g.n, k),
            size.cpu().numpy().view(np.uint32), est.cpu().numpy(), ranks, size)


def _check(oracle_lib, g, ell, k, seed, queries=0):
    import torch
    import paper_1408_6282_amd as sk
    R, S, E, rt, st = _build(g, ell, k, seed)
    R0, S0, _ = oracle_lib.build_alg2_perm(g, seed, ell, k)
    assert np.array_equal(S, S0), "sizes differ"
    assert np.array_equal(R, R0), "sketches differ"
    assert np.array_equal(E, oracle_lib.perm_estimates(R0, S0, g.n, k, ell)), "estimates differ"
    if queries:
        off, nodes = uniform_query_sets(queries, g.n, seed % 1000, 1, min(64, g.n))
        est = torch.empty(queries, dtype=torch.float64, device=dev())
        status = torch.empty(queries, dtype=torch.int32, device=dev())
        for estimator in (0, 1):
            sk.skim_perm_query_batch(rt, st, g.n, k, ell, to_dev_u64(off), to_dev_u32(nodes), est,
                                     status, estimator=estimator)
            torch.cuda.synchronize()
            want, wst = oracle_lib.perm_union_query(R0, S0, g.n, k, ell, off, nodes, estimator)
            assert np.array_equal(est.cpu().numpy(), want), f"estimator {estimator}"
            assert np.array_equal(status.cpu().numpy(), wst)


@pytest.mark.parametrize("ell,k", [(1, 2), (4, 16), (16, 4), (16, 16), (64, 64), (7, 5), (64, 256)])
def test_random_small_graphs(oracle_lib, ell, k):
    rng = np.random.default_rng(500 + ell * 7 + k)
    for trial in range(4):
        n = int(rng.integers(2, 60))
        src, dst, thr = random_small_graph(rng, n, int(rng.integers(0, 4 * n)),
                                           [U32, U32 // 2, U32 // 4, U32 // 20])
        g = from_edges(n, src, dst, thr if len(src) else None)
        seed = int(rng.integers(0, 2 ** 63))
        log(f"perm ell={ell} k={k} n={n} m={g.m} seed={seed}")
        _check(oracle_lib, g, ell, k, seed, queries=200)


def test_p1_and_edgeless(oracle_lib):
    rng = np.random.default_rng(9)
    src, dst, _ = random_small_graph(rng, 40, 100, [U32])
    _check(oracle_lib, from_edges(40, src, dst, U32), 16, 8, 3, queries=100)
    _check(oracle_lib, from_edges(40, [], []), 16, 8, 3, queries=100)


@pytest.mark.parametrize("name", ["tiny-ic", "served-skim"])
def test_configs(oracle_lib, name):
    cfg = make_config(name)
    _check(oracle_lib, make_graph(cfg), cfg["ell"], cfg["k"], cfg["seed"], queries=2000)


def test_chung_lu_20k_wc(oracle_lib):
    from workloads.graphs import Graph, chung_lu_graph, wc_thresholds
    n = 20000
    rp, col = chung_lu_graph(n, 320000, 2.1, 57)
    g = Graph(n, rp, col, wc_thresholds(rp, col, n))
    for ell, k in [(64, 64), (64, 16)]:
        log(f"chung-lu 20k wc, l={ell} k={k}")
        _check(oracle_lib, g, ell, k, 11, queries=1000)


def test_pull_levels(oracle_lib):
    # every search level by pull, and pull from 300 entries: the positions'
    # sketches are those of the push (the same visits in another order)
    import paper_1408_6282_amd as sk
    from workloads.graphs import Graph, chung_lu_graph, wc_thresholds
    n = 20000
    rp, col = chung_lu_graph(n, 320000, 2.1, 57)
    g = Graph(n, rp, col, wc_thresholds(rp, col, n))
    rng = np.random.default_rng(31)
    src, dst, thr = random_small_graph(rng, 50, 200, [U32, U32 // 3])
    small = from_edges(50, src, dst, thr)
    try:
        for pull in (1, 300):
            sk.skim_set_build_params(dict(pull_frontier=pull))
            log(f"perm, pull from {pull} entries")
            _check(oracle_lib, g, 64, 16, 11)
            _check(oracle_lib, small, 16, 8, 5)
    finally:
        sk.skim_set_build_params(None)
