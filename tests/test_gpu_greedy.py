"""GPU parity of skim_greedy against the oracle's Algorithm 1: bit-exact seed
sequences and newly-covered pair counts, resumed runs equal to one-shot runs,
the exhaustion (exact-greedy) regime, and the served-SKIM configuration."""
import numpy as np
import pytest

from workloads import from_edges
from workloads.configs import make_config, make_graph
from brute import random_small_graph
from gpu_util import gpu_greedy, log

pytestmark = pytest.mark.gpu


def test_served_skim_config_200_seeds(oracle_lib):
    cfg = make_config("served-skim")
    g = make_graph(cfg)
    log("served-skim 200 seeds one-shot")
    seeds, gains, gd, sel = gpu_greedy(g, cfg["ell"], cfg["k"], cfg["seed"], [200])
    ws, wg, _ = oracle_lib.skim(g, cfg["seed"], cfg["ell"], cfg["k"], 200)
    assert np.array_equal(seeds, ws)
    assert np.array_equal(gains, wg)
    assert np.array_equal(gd, wg.astype(np.float64) / cfg["ell"])
    assert sel == 200
    log("served-skim 4 x 50 resumed")
    s2, g2, _, _ = gpu_greedy(g, cfg["ell"], cfg["k"], cfg["seed"], [50, 50, 50, 50])
    assert np.array_equal(s2, seeds) and np.array_equal(g2, gains)


@pytest.mark.parametrize("ell,k", [(1, 2), (4, 3), (16, 8), (64, 64)])
def test_random_graphs(oracle_lib, ell, k):
    rng = np.random.default_rng(ell * 7 + k)
    for trial in range(4):
        n = int(rng.integers(2, 80))
        src, dst, thr = random_small_graph(rng, n, int(rng.integers(0, 3 * n)),
                                           [0xFFFFFFFF, 0xFFFFFFFF // 2, 0xFFFFFFFF // 10])
        g = from_edges(n, src, dst, thr)
        seed = int(rng.integers(0, 2 ** 62))
        s = int(rng.integers(1, n + 1))
        log(f"skim ell={ell} k={k} n={n} m={g.m} s={s} seed={seed}")
        seeds, gains, _, _ = gpu_greedy(g, ell, k, seed, [s])
        ws, wg, _ = oracle_lib.skim(g, seed, ell, k, s)
        assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)


def test_exhaustion_full_permutation(oracle_lib):
    rng = np.random.default_rng(4)
    n = 60
    src, dst, thr = random_small_graph(rng, n, 150, [0xFFFFFFFF // 2])
    g = from_edges(n, src, dst, thr)
    ell, k = 8, 10_000  # no sketch ever fills: every seed by the exhaustion rule
    seeds, gains, _, _ = gpu_greedy(g, ell, k, 7, [20, 40])
    ws, wg, cnt = oracle_lib.skim(g, 7, ell, k, n)
    assert cnt["fallback"] == n
    assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)
    assert int(gains.sum()) == n * ell


def test_too_many_seeds_rejected():
    import torch
    import paper_1408_6282_amd as sk
    g = from_edges(5, [0, 1], [1, 2])
    G = sk.DeviceGraph.from_host(g, "cuda:0")
    a = torch.empty(6, dtype=torch.int32, device="cuda:0")
    b = torch.empty(6, dtype=torch.int64, device="cuda:0")
    with pytest.raises(sk.SkimError) as ei:
        sk.skim_greedy(G, 4, 4, 1, 6, a, b)
    assert ei.value.status == sk.SKIM_EINVAL
    # sizes and batch counters are 16-bit halves of words: k <= 65535
    for ell, k in [(4, 65536), (65, 4), (4, 1)]:
        with pytest.raises(sk.SkimError) as ei:
            sk.skim_greedy(G, ell, k, 1, 2, a, b)
        assert ei.value.status == sk.SKIM_EINVAL


def test_weighted_cascade_20k(oracle_lib):
    # heavy-tailed reach: seeds whose residual searches cover thousands of pairs
    from workloads.graphs import Graph, chung_lu_graph, wc_thresholds
    n = 20000
    rp, col = chung_lu_graph(n, 320000, 2.1, 56)
    g = Graph(n, rp, col, wc_thresholds(rp, col, n))
    for ell, k, s in ((16, 16, 20), (64, 64, 30)):
        log(f"skim chung-lu 20k wc ell={ell} k={k} s={s}")
        seeds, gains, _, _ = gpu_greedy(g, ell, k, 1, [s])
        ws, wg, _ = oracle_lib.skim(g, 1, ell, k, s)
        assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)


def test_counters_outside_lds(oracle_lib):
    # more nodes than the LDS copy of the counters holds: they stay in global memory
    from workloads.graphs import Graph, er_graph
    n = 30000
    rp, col = er_graph(n, 150000, 71)
    g = Graph(n, rp, col, np.full(col.size, 0xFFFFFFFF // 8, dtype=np.uint32))
    log("skim ER 30k p=1/8 ell=8 k=8 s=12")
    seeds, gains, _, _ = gpu_greedy(g, 8, 8, 3, [5, 7])
    ws, wg, _ = oracle_lib.skim(g, 3, 8, 8, 12)
    assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)


@pytest.mark.slow
def test_chung_lu_1m_equals_oracle():
    # SKIM on the 1M-node weighted-cascade graph (l = k = 64), 50 seeds in two
    # resumed calls, against the oracle's sequence stored by
    # tests/golden/make_skim.py (single-threaded Algorithm 1)
    import json
    import os
    from workloads.configs import graph_sha256, make_config, make_graph
    from gpu_util import log
    cfg = make_config("chung-lu-1m")
    g = make_graph(cfg)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "chung_lu_1m_skim.json")
    with open(path) as f:
        gold = json.load(f)
    assert gold["graph_sha256"] == graph_sha256(g)
    log("gpu SKIM on chung-lu-1m")
    seeds, gains, _, _ = gpu_greedy(g, cfg["ell"], cfg["k"], cfg["seed"], [20, 30])
    assert seeds.tolist() == gold["seeds"]
    assert gains.tolist() == gold["gain_pairs"]


@pytest.mark.parametrize("ell,k", [(16, 8), (64, 16)])
def test_hub_seed_residual_on_the_grid(oracle_lib, ell, k):
    # a hub with 20,000 out-edges at p = 0.3 over leaves joined by p = 1/8
    # edges: the first seed is the hub, whose residual search is handed to the
    # whole grid at its first level (thousands of live out-edges per instance,
    # expanded edge-balanced), then the loop resumes in the workgroup with the
    # sizes the grid left; later seeds are small
    rng = np.random.default_rng(91)
    leaves = 20000
    n = 1 + leaves
    src, dst = [0] * leaves, list(range(1, n))
    thr = [int(0xFFFFFFFF * 0.3)] * leaves
    seen = set(zip(src, dst))
    for a, b in zip(rng.integers(1, n, 40000).tolist(), rng.integers(1, n, 40000).tolist()):
        if a != b and (a, b) not in seen:
            seen.add((a, b))
            src.append(a)
            dst.append(b)
            thr.append(0xFFFFFFFF // 8)
    g = from_edges(n, src, dst, thr)
    seeds, gains, _, _ = gpu_greedy(g, ell, k, 3, [5, 7])
    ws, wg, _ = oracle_lib.skim(g, 3, ell, k, 12)
    assert seeds[0] == 0
    assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)


def _run(sk, G, ell, k, seed, state, s):
    import torch
    d = torch.device("cuda:0")
    a = torch.empty(s, dtype=torch.int32, device=d)
    b = torch.empty(s, dtype=torch.int64, device=d)
    sk.skim_greedy(G, ell, k, seed, s, a, b, state=state)
    torch.cuda.synchronize()
    return a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint64)


def _records(sk, state):
    import torch
    d = torch.device("cuda:0")
    s = state.selected
    tau = torch.empty(s, dtype=torch.int64, device=d)
    sec = torch.empty(s, dtype=torch.int32, device=d)
    sk.skim_greedy_records(state, 0, s, tau, sec)
    torch.cuda.synchronize()
    return tau.cpu().numpy().view(np.uint64), sec.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("name,first,rest", [("served-skim", 70, 130), ("wc-20k", 20, 30)])
def test_state_saved_and_loaded_resumes_the_run(oracle_lib, name, first, rest):
    # a run suspended after `first` seeds, saved to host bytes, freed, loaded
    # into a new state and resumed gives the oracle's sequence, gains and
    # per-seed error records for all first + rest seeds
    import paper_1408_6282_amd as sk
    import torch
    if name == "served-skim":
        cfg = make_config("served-skim")
        g, ell, k, seed = make_graph(cfg), cfg["ell"], cfg["k"], cfg["seed"]
    else:
        from workloads.graphs import Graph, chung_lu_graph, wc_thresholds
        rp, col = chung_lu_graph(20000, 320000, 2.1, 56)
        g, ell, k, seed = Graph(20000, rp, col, wc_thresholds(rp, col, 20000)), 64, 64, 1
    G = sk.DeviceGraph.from_host(g, torch.device("cuda:0"))
    a = sk.GreedyState()
    try:
        s1, g1 = _run(sk, G, ell, k, seed, a, first)
        data = a.save()
        log(f"{name}: saved after {first} seeds, {len(data)} bytes")
    finally:
        a.free()
    b = sk.GreedyState.load(G, ell, k, seed, data)
    try:
        assert b.selected == first
        s2, g2 = _run(sk, G, ell, k, seed, b, rest)
        tau, sec = _records(sk, b)
    finally:
        b.free()
    ws, wg, wt, wsec, _ = oracle_lib.skim(g, seed, ell, k, first + rest, records=True)
    assert np.array_equal(np.concatenate([s1, s2]), ws)
    assert np.array_equal(np.concatenate([g1, g2]), wg)
    assert np.array_equal(tau, wt) and np.array_equal(sec, wsec)


def test_saved_state_refused_for_other_runs():
    import paper_1408_6282_amd as sk
    import torch
    cfg = make_config("tiny-ic")
    g = make_graph(cfg)
    G = sk.DeviceGraph.from_host(g, torch.device("cuda:0"))
    a = sk.GreedyState()
    try:
        _run(sk, G, 8, 4, 3, a, 5)
        data = a.save()
    finally:
        a.free()
    for ell, k, seed, blob in ((8, 5, 3, data), (8, 4, 4, data), (16, 4, 3, data),
                               (8, 4, 3, data[:-8]), (8, 4, 3, b"x" * len(data))):
        with pytest.raises(sk.SkimError) as ei:
            sk.GreedyState.load(G, ell, k, seed, blob)
        assert ei.value.status == sk.SKIM_EINVAL
    b = sk.GreedyState.load(G, 8, 4, 3, data)  # the right parameters load
    try:
        assert b.selected == 5
    finally:
        b.free()
