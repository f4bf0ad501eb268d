"""GPU parity of skim_build_sketches against the CPU oracle (bit-exact sketches,
sizes and estimates), on random small graphs, the tiny config, a mid-size
power-law graph spanning many rank windows, edge cases, invalid inputs, and
the full 1M-node Chung-Lu configuration."""
import numpy as np
import pytest

from workloads import from_edges
from workloads.configs import make_config, make_graph
from brute import random_small_graph
from gpu_util import gpu_build, log

pytestmark = pytest.mark.gpu

THRS = [0xFFFFFFFF, 0xFFFFFFFF // 2, 0xFFFFFFFF // 4, 0xFFFFFFFF // 20]


def _check(oracle_lib, g, ell, k, seed):
    R, S, E, work, _ = gpu_build(g, ell, k, seed)
    R0, S0, _ = oracle_lib.build_alg2(g, seed, ell, k)
    E0 = oracle_lib.estimates(R0, S0, k, ell)
    assert np.array_equal(R, R0), "sketch ranks differ"
    assert np.array_equal(S, S0), "sketch sizes differ"
    assert np.array_equal(E, E0), "estimates differ"  # IEEE, same operation order
    return work


@pytest.mark.parametrize("ell,k", [(1, 2), (2, 3), (16, 4), (16, 16), (64, 64), (7, 5), (64, 256)])
def test_random_small_graphs(oracle_lib, ell, k):
    rng = np.random.default_rng(1000 * ell + k)
    for trial in range(6):
        n = int(rng.integers(1, 60))
        m = int(rng.integers(0, 4 * n)) if n > 1 else 0
        src, dst, thr = random_small_graph(rng, n, m, THRS) if n > 1 else ([], [], [])
        g = from_edges(n, src, dst, thr if len(src) else None)
        seed = int(rng.integers(0, 2 ** 63))
        log(f"random graph ell={ell} k={k} trial={trial} n={n} m={g.m} seed={seed}")
        _check(oracle_lib, g, ell, k, seed)


def test_tiny_config(oracle_lib):
    cfg = make_config("tiny-ic")
    g = make_graph(cfg)
    log("tiny-ic")
    work = _check(oracle_lib, g, cfg["ell"], cfg["k"], cfg["seed"])
    assert work["windows"] >= 1


def test_deterministic_graph_and_no_edges(oracle_lib):
    rng = np.random.default_rng(3)
    src, dst, _ = random_small_graph(rng, 200, 900, [0xFFFFFFFF])
    log("p=1 graph")
    _check(oracle_lib, from_edges(200, src, dst, 0xFFFFFFFF), 8, 16, 5)
    log("no edges")
    _check(oracle_lib, from_edges(300, [], []), 16, 8, 6)


def test_deep_path_many_levels(oracle_lib):
    # a p=1 path of 3000 nodes: reverse searches 3000 levels deep
    n = 3000
    g = from_edges(n, list(range(n - 1)), list(range(1, n)), 0xFFFFFFFF)
    log("deep path")
    _check(oracle_lib, g, 4, 8, 11)


def test_powerlaw_many_windows(oracle_lib):
    from workloads.graphs import Graph, chung_lu_graph, wc_thresholds
    rp, col = chung_lu_graph(20000, 320000, 2.1, 55)
    g = Graph(20000, rp, col, wc_thresholds(rp, col, 20000))
    log("chung-lu 20k wc l=64 k=64")
    work = _check(oracle_lib, g, 64, 64, 1)
    log(f"work {work}")
    assert work["windows"] >= 4 and work["restarts"] == 0
    log("chung-lu 20k uniform p=0.1 l=32 k=16")
    g2 = Graph(20000, rp, col, np.full(col.size, 0xFFFFFFFF // 10, dtype=np.uint32))
    _check(oracle_lib, g2, 32, 16, 2)


def test_hub_lists_spread_over_the_grid(oracle_lib):
    # live in-lists longer than 4096 entries (a p = 1 in-star of 6000
    # leaves into a hub, the hub feeding a chain, plus random p = 1/2 edges):
    # the searches from the chain visit the hub and expand its list on the
    # whole grid (k_expand_heavy) as well as in the tails and levels
    rng = np.random.default_rng(77)
    leaves, chain = 6000, 300
    n = 1 + leaves + chain
    src = list(range(1, leaves + 1)) + [0] + list(range(leaves + 1, n - 1))
    dst = [0] * leaves + [leaves + 1] + list(range(leaves + 2, n))
    thr = [0xFFFFFFFF] * len(src)
    extra = 20000
    es, ed = rng.integers(0, n, extra), rng.integers(0, n, extra)
    seen = set(zip(src, dst))
    for a, b in zip(es.tolist(), ed.tolist()):
        if a != b and (a, b) not in seen:
            seen.add((a, b))
            src.append(a)
            dst.append(b)
            thr.append(0xFFFFFFFF // 2)
    g = from_edges(n, src, dst, thr)
    for ell, k, seed in ((64, 16, 5), (8, 64, 6)):
        log(f"hub lists n={n} m={g.m} l={ell} k={k}")
        _check(oracle_lib, g, ell, k, seed)


def test_medium_lists_spread_over_the_workgroup(oracle_lib):
    # live in-lists of 17 to 4096 sources (p = 1 in-stars of 20 to 3000
    # leaves into 12 hubs that feed each other) next to short random lists:
    # a workgroup lays a chunk's long lists end to end, a wave its entries'
    # short ones
    rng = np.random.default_rng(78)
    sizes = [20, 33, 64, 100, 257, 300, 511, 700, 1000, 1500, 2048, 3000]
    hubs = len(sizes)
    n = hubs + sum(sizes)
    src, dst, thr = [], [], []
    nxt = hubs
    for h, sz in enumerate(sizes):
        for leaf in range(nxt, nxt + sz):
            src.append(leaf)
            dst.append(h)
            thr.append(0xFFFFFFFF)
        nxt += sz
        src.append(h)
        dst.append((h + 1) % hubs)
        thr.append(0xFFFFFFFF // 2)
    seen = set(zip(src, dst))
    for a, b in zip(rng.integers(0, n, 3 * n).tolist(), rng.integers(0, n, 3 * n).tolist()):
        if a != b and (a, b) not in seen:
            seen.add((a, b))
            src.append(a)
            dst.append(b)
            thr.append(0xFFFFFFFF // 3)
    g = from_edges(n, src, dst, thr)
    for ell, k, seed in ((64, 16, 8), (16, 64, 9)):
        log(f"medium lists n={n} m={g.m} l={ell} k={k}")
        _check(oracle_lib, g, ell, k, seed)


def test_deterministic_repeat():
    cfg = make_config("tiny-ic")
    g = make_graph(cfg)
    a = gpu_build(g, 16, 16, 1)
    b = gpu_build(g, 16, 16, 1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("bad", ["unsorted", "duplicate", "self_loop", "head_range", "row_ptr"])
def test_invalid_graph_rejected(bad):
    import torch
    import paper_1408_6282_amd as sk
    from workloads.graphs import Graph
    rp = np.array([0, 2, 3, 3], dtype=np.uint64)
    col = np.array([1, 2, 2], dtype=np.uint32)
    if bad == "unsorted":
        col = np.array([2, 1, 2], dtype=np.uint32)
    elif bad == "duplicate":
        col = np.array([1, 1, 2], dtype=np.uint32)
    elif bad == "self_loop":
        col = np.array([0, 2, 2], dtype=np.uint32)
    elif bad == "head_range":
        col = np.array([1, 7, 2], dtype=np.uint32)
    elif bad == "row_ptr":
        rp = np.array([0, 3, 2, 3], dtype=np.uint64)
    g = Graph(3, rp, col, np.full(3, 0xFFFFFFFF, dtype=np.uint32))
    G = sk.DeviceGraph.from_host(g, "cuda:0")
    ranks = torch.full((3 * 4,), 7, dtype=torch.int64, device="cuda:0")
    size = torch.full((3,), 7, dtype=torch.int32, device="cuda:0")
    with pytest.raises(sk.SkimError) as ei:
        sk.skim_build_sketches(G, 4, 4, 1, ranks, size)
    assert ei.value.status == sk.SKIM_EINVAL
    assert (ranks.cpu() == 7).all() and (size.cpu() == 7).all()  # outputs untouched


def test_bad_parameters():
    import torch
    import paper_1408_6282_amd as sk
    g = from_edges(4, [0], [1])
    G = sk.DeviceGraph.from_host(g, "cuda:0")
    ranks = torch.empty(4 * 4, dtype=torch.int64, device="cuda:0")
    size = torch.empty(4, dtype=torch.int32, device="cuda:0")
    for ell, k in [(0, 4), (65, 4), (4, 1), (4, 257)]:
        with pytest.raises(sk.SkimError) as ei:
            sk.skim_build_sketches(G, ell, k, 1, ranks, size)
        assert ei.value.status == sk.SKIM_EINVAL


# Launch shapes of the full-size parity runs: the defaults, the shapes the
# autotuner picks on this workload (the launch the bench times), the widest
# windows and batches, every level by pull, and pull from 2^21 entries.
CL_SHAPES = {
    "default": None,
    "tuned": dict(small_frontier=262144, small_batch=16, large_batch=2, thread_frontier=524288,
                  heavy_visits=4, sort_frontier=0, window_span=3, first_span=5),
    "wide": dict(small_frontier=1 << 24, small_batch=64, large_batch=64, thread_frontier=1 << 30,
                 heavy_visits=1000, sort_frontier=0, window_span=8, first_span=16),
    "pull": dict(pull_frontier=1),
    "pull-2m": dict(pull_frontier=1 << 21),
}


@pytest.fixture(scope="module")
def chung_lu_1m():
    cfg = make_config("chung-lu-1m")
    log("generating chung-lu-1m")
    return cfg, make_graph(cfg)


@pytest.mark.slow
@pytest.mark.parametrize("shape", list(CL_SHAPES))
def test_chung_lu_1m_full_parity(chung_lu_1m, shape):
    # every sketch, size and estimate of the full workload equals the
    # oracle's Algorithm 2 (by the digests its committed script stored)
    import paper_1408_6282_amd as sk
    from gpu_util import check_digests, golden
    cfg, g = chung_lu_1m
    sk.skim_set_build_params(CL_SHAPES[shape])
    try:
        log(f"gpu build chung-lu-1m, {shape} shapes")
        R, S, E, work, _ = gpu_build(g, cfg["ell"], cfg["k"], cfg["seed"])
    finally:
        sk.skim_set_build_params(None)
    log(f"gpu work {work}")
    check_digests(golden("chung_lu_1m"), g, R, S, E)
