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
