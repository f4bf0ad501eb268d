"""GPU parity of skim_build_ic_sketches (Section 3, sketches for an IC model
with structured permutation ranks) against the oracle: every position and
every estimate bit for bit (the estimate is one correctly rounded division
of the same operands on both sides).

Cases: the served-SKIM and tiny-IC configurations; random small graphs over k
with p = 1, no edges and mixed probabilities; an Erdos-Renyi graph and a
weighted-cascade Chung-Lu graph of 20,000 nodes; invalid parameters.
"""
import numpy as np
import pytest

from workloads import from_edges
from workloads.configs import make_config, make_graph
from brute import random_small_graph
from gpu_util import dev, log

pytestmark = pytest.mark.gpu


def gpu_ic(g, k, seed):
    import torch
    import paper_1408_6282_amd as sk
    G = sk.DeviceGraph.from_host(g, dev())
    pos = torch.zeros(g.n * k, dtype=torch.int32, device=dev())
    est = torch.full((g.n,), -1.0, dtype=torch.float64, device=dev())
    sk.skim_build_ic_sketches(G, k, seed, pos, est)
    torch.cuda.synchronize()
    return pos.cpu().numpy().view(np.uint32).reshape(g.n, k), est.cpu().numpy()


def _check(oracle_lib, g, k, seed):
    pos, est = gpu_ic(g, k, seed)
    wpos, west, _ = oracle_lib.ic_sketches(g, k, seed)
    assert np.array_equal(pos, wpos)
    assert np.array_equal(est, west)


def test_configs(oracle_lib):
    for name, k in (("served-skim", 64), ("tiny-ic", 16)):
        cfg = make_config(name)
        g = make_graph(cfg)
        log(f"ic sketches {name} k={k}")
        _check(oracle_lib, g, k, cfg["seed"])


@pytest.mark.parametrize("k", [2, 5, 32, 256])
def test_random_small_graphs(oracle_lib, k):
    rng = np.random.default_rng(k + 900)
    for trial in range(4):
        n = int(rng.integers(1, 90))
        src, dst, thr = random_small_graph(rng, n, int(rng.integers(0, 4 * n + 1)),
                                           [0xFFFFFFFF, 0xFFFFFFFF // 2, 0xFFFFFFFF // 10])
        g = from_edges(n, src, dst, thr)
        seed = int(rng.integers(0, 2 ** 63))
        log(f"ic k={k} n={n} m={g.m} seed={seed}")
        _check(oracle_lib, g, k, seed)
    _check(oracle_lib, from_edges(7, [], []), k, 3)                                  # no edges
    _check(oracle_lib, from_edges(6, [0, 1, 2, 3, 4], [1, 2, 3, 4, 5], 0xFFFFFFFF), k, 4)  # p = 1


def test_20k_graphs(oracle_lib):
    from workloads.graphs import Graph, chung_lu_graph, er_graph, wc_thresholds
    rp, col = er_graph(20000, 160000, 31)
    g = Graph(20000, rp, col, np.full(col.size, 0xFFFFFFFF // 100, dtype=np.uint32))
    log("ic ER 20k p=0.01 k=16")
    _check(oracle_lib, g, 16, 5)
    rp, col = chung_lu_graph(20000, 320000, 2.1, 56)
    g = Graph(20000, rp, col, wc_thresholds(rp, col, 20000))
    log("ic chung-lu 20k wc k=8")
    _check(oracle_lib, g, 8, 6)


def test_bad_parameters():
    import torch
    import paper_1408_6282_amd as sk
    g = from_edges(5, [0, 1], [1, 2])
    G = sk.DeviceGraph.from_host(g, dev())
    pos = torch.zeros(5 * 300, dtype=torch.int32, device=dev())
    for k in (0, 1, 257):
        with pytest.raises(sk.SkimError) as ei:
            sk.skim_build_ic_sketches(G, k, 1, pos)
        assert ei.value.status == sk.SKIM_EINVAL
    with pytest.raises(sk.SkimError) as ei:
        sk.skim_build_ic_sketches(G, 4, 1, None)
    assert ei.value.status == sk.SKIM_EINVAL


def gpu_ic_query(pos_t, n, k, off, nodes, estimator):
    import torch
    import paper_1408_6282_amd as sk
    from gpu_util import to_dev_u32, to_dev_u64
    q = len(off) - 1
    est = torch.full((max(q, 1),), -9.0, dtype=torch.float64, device=dev())
    st = torch.full((max(q, 1),), 9, dtype=torch.int32, device=dev())
    sk.skim_ic_query_batch(pos_t, n, k, to_dev_u64(off), to_dev_u32(nodes) if len(nodes) else None,
                           est, st, estimator=estimator)
    torch.cuda.synchronize()
    return est.cpu().numpy()[:q], st.cpu().numpy()[:q]


@pytest.mark.parametrize("name,k", [("served-skim", 64), ("tiny-ic", 16)])
def test_union_queries(oracle_lib, name, k):
    import torch
    from workloads import uniform_query_sets
    cfg = make_config(name)
    g = make_graph(cfg)
    pos, _ = gpu_ic(g, k, cfg["seed"])
    pos_t = torch.from_numpy(pos.view(np.int32).reshape(-1).copy()).to(dev())
    off, nodes = uniform_query_sets(3000, g.n, 41, 1, 512)
    # extra cases: empty, duplicates, an invalid node, more than 1024 members
    extra = [[], [5, 5, 9, 5], [3, g.n], list(range(g.n)) * 2]  # the last: 2000 members
    sizes = np.diff(off.astype(np.int64)).tolist() + [len(e) for e in extra]
    nodes = np.concatenate([nodes, np.array([v for e in extra for v in e], dtype=np.uint32)])
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    for estimator in (0, 1):
        log(f"ic union queries {name} estimator={estimator}")
        est, st = gpu_ic_query(pos_t, g.n, k, off, nodes, estimator)
        west, wst = oracle_lib.ic_union_query(pos, g.n, k, off, nodes, estimator)
        assert st[-1] == -2 and est[-1] == 0.0
        assert np.array_equal(st[:-1], wst[:-1])
        assert np.array_equal(est[:-1], west[:-1])


def test_union_query_errors():
    import torch
    import paper_1408_6282_amd as sk
    from gpu_util import to_dev_u32, to_dev_u64
    pos = torch.ones(10 * 4, dtype=torch.int32, device=dev())
    est = torch.empty(2, dtype=torch.float64, device=dev())
    nodes = to_dev_u32([0, 1])
    for kw in ({"k": 1}, {"k": 257}, {"estimator": 2}):
        k = kw.get("k", 4)
        with pytest.raises(sk.SkimError) as ei:
            sk.skim_ic_query_batch(pos, 10, k, to_dev_u64([0, 1, 2]), nodes, est,
                                   estimator=kw.get("estimator", 0))
        assert ei.value.status == sk.SKIM_EINVAL
    for off in ([1, 1, 2], [0, 2, 1]):
        with pytest.raises(sk.SkimError) as ei:
            sk.skim_ic_query_batch(pos, 10, 4, to_dev_u64(off), nodes, est)
        assert ei.value.status == sk.SKIM_EINVAL


def test_searches_handed_to_workgroups(oracle_lib):
    # p = 1: a 3000-node path (position t's search reaches every predecessor
    # of v_t) and a random graph whose giant component exceeds 1024 nodes,
    # so most searches outgrow a thread's queue and go to the workgroup path
    from workloads.graphs import Graph, er_graph
    n = 3000
    log("ic path 3000 p=1 k=4")
    _check(oracle_lib, from_edges(n, list(range(n - 1)), list(range(1, n)), 0xFFFFFFFF), 4, 12)
    rp, col = er_graph(2500, 10000, 61)
    g = Graph(2500, rp, col, np.full(col.size, 0xFFFFFFFF, dtype=np.uint32))
    log("ic ER 2500 p=1 k=3")
    _check(oracle_lib, g, 3, 13)
    rp, col = er_graph(4000, 12000, 62)
    g = Graph(4000, rp, col, np.full(col.size, 0xFFFFFFFF // 2, dtype=np.uint32))
    log("ic ER 4000 p=1/2 k=5")
    _check(oracle_lib, g, 5, 14)


def test_counting_path(oracle_lib):
    # builds whose single appending pass runs out of room (forced by the
    # host-side hook) count first and write after, with the same results,
    # also with searches handed to workgroups
    import paper_1408_6282_amd as sk
    from workloads.graphs import Graph, er_graph, chung_lu_graph, wc_thresholds
    rp, col = chung_lu_graph(20000, 320000, 2.1, 58)
    cases = [(Graph(20000, rp, col, wc_thresholds(rp, col, 20000)), 8, 15)]
    rp, col = er_graph(2500, 10000, 61)
    cases.append((Graph(2500, rp, col, np.full(col.size, 0xFFFFFFFF, dtype=np.uint32)), 3, 13))
    try:
        for g, k, seed in cases:
            log(f"ic counting path n={g.n} k={k}")
            sk.skim_debug_inject(sk.SKIM_FAULT_IC_RECORDS, 1)
            _check(oracle_lib, g, k, seed)
    finally:
        sk.skim_debug_inject(sk.SKIM_FAULT_IC_RECORDS, 0)
