"""Launch shapes of the sketch build (skim_build_params) and their autotuner:
any valid shape gives the oracle's sketches bit for bit, the tuner leaves the
fastest shape in force, and out-of-range shapes are refused."""
import numpy as np
import pytest

from workloads import from_edges
from brute import random_small_graph
from gpu_util import gpu_build, log

pytestmark = pytest.mark.gpu

EXTREME = dict(small_frontier=1, small_batch=1, large_batch=1, thread_frontier=1, heavy_visits=1,
               sort_frontier=1, window_span=1, first_span=1)
WIDE = dict(small_frontier=1 << 24, small_batch=64, large_batch=64, thread_frontier=1 << 30,
            heavy_visits=1000, sort_frontier=0, window_span=8, first_span=16)
# every level by pull, and pull only for levels of 300 entries or more (a
# window's levels then change direction as its frontier grows and shrinks)
SHAPES = {"extreme": EXTREME, "wide": WIDE, "pull": dict(pull_frontier=1),
          "mixed": dict(pull_frontier=300)}


@pytest.fixture
def restore_params():
    import paper_1408_6282_amd as sk
    yield
    sk.skim_set_build_params(None)


def _powerlaw(n=20000, m=320000):
    from workloads.graphs import Graph, chung_lu_graph, wc_thresholds
    rp, col = chung_lu_graph(n, m, 2.1, 55)
    return Graph(n, rp, col, wc_thresholds(rp, col, n))


@pytest.mark.parametrize("shape", list(SHAPES))
def test_any_shape_gives_oracle_sketches(oracle_lib, restore_params, shape):
    import paper_1408_6282_amd as sk
    sk.skim_set_build_params(SHAPES[shape])
    rng = np.random.default_rng(5)
    graphs = [_powerlaw()]
    for _ in range(3):
        src, dst, thr = random_small_graph(rng, 50, 200, [0xFFFFFFFF, 0xFFFFFFFF // 3])
        graphs.append(from_edges(50, src, dst, thr))
    for g in graphs:
        log(f"shape {shape}: n={g.n} m={g.m}")
        R, S, E, work, _ = gpu_build(g, 32, 16, 3)
        R0, S0, _ = oracle_lib.build_alg2(g, 3, 32, 16)
        assert np.array_equal(R, R0) and np.array_equal(S, S0)
        assert np.array_equal(E, oracle_lib.estimates(R0, S0, 16, 32))


def test_tuner_keeps_results_and_sets_params(oracle_lib, restore_params):
    import torch
    import paper_1408_6282_amd as sk
    g = _powerlaw()
    G = sk.DeviceGraph.from_host(g, "cuda:0")
    ranks = torch.empty(g.n * 16, dtype=torch.int64, device="cuda:0")
    size = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    best, best_ms, start_ms = sk.skim_tune_build(G, 32, 16, 3, ranks, size, reps=1)
    log(f"tuned {best} {best_ms:.3f} ms (start {start_ms:.3f} ms)")
    assert best_ms <= start_ms
    assert sk.skim_get_build_params() == best
    R0, S0, _ = oracle_lib.build_alg2(g, 3, 32, 16)
    R = ranks.cpu().numpy().view(np.uint64).reshape(g.n, 16)
    assert np.array_equal(R, R0) and np.array_equal(size.cpu().numpy().view(np.uint32), S0)


@pytest.mark.parametrize("field,value", [("small_frontier", 0), ("small_batch", 0),
                                         ("small_batch", 65), ("large_batch", 0),
                                         ("thread_frontier", 0), ("heavy_visits", 0),
                                         ("window_span", 0), ("window_span", 9),
                                         ("first_span", 0), ("first_span", 17)])
def test_out_of_range_params_refused(restore_params, field, value):
    import paper_1408_6282_amd as sk
    before = sk.skim_get_build_params()
    with pytest.raises(sk.SkimError) as ei:
        sk.skim_set_build_params({field: value})
    assert ei.value.status == sk.SKIM_EINVAL
    assert sk.skim_get_build_params() == before


def test_tuning_cache(tmp_path):
    import torch
    import paper_1408_6282_amd as sk
    from workloads.configs import make_config, make_graph
    cfg = make_config("tiny-ic")
    g = make_graph(cfg)
    G = sk.DeviceGraph.from_host(g, "cuda:0")
    ranks = torch.empty(g.n * 16, dtype=torch.int64, device="cuda:0")
    size = torch.empty(g.n, dtype=torch.int32, device="cuda:0")
    path = str(tmp_path / "tune.txt")
    try:
        p1, ms1, _, hit1 = sk.skim_tune_build_cached(G, 16, 16, 1, ranks, size, path, reps=1)
        assert not hit1
        lines = open(path).read().splitlines()
        assert len(lines) == 1 and len(lines[0].split()) == 11  # key, 9 shapes, time
        sk.skim_set_build_params(None)
        p2, ms2, start2, hit2 = sk.skim_tune_build_cached(G, 16, 16, 1, ranks, size, path, reps=1)
        assert hit2 and p2 == p1 and start2 == 0.0
        assert sk.skim_get_build_params() == p1  # the stored shapes are in force
        # another configuration (k), another key; a garbage line is skipped
        with open(path, "a") as f:
            f.write("not a cache line\n")
        _, _, _, hit3 = sk.skim_tune_build_cached(G, 16, 8, 1, ranks, size, path, reps=1)
        assert not hit3 and len(open(path).read().splitlines()) == 3
        _, _, _, hit4 = sk.skim_tune_build_cached(G, 16, 8, 1, ranks, size, path, reps=1)
        assert hit4
        with pytest.raises(sk.SkimError):
            sk.skim_tune_build_cached(G, 16, 16, 1, ranks, size, "", reps=1)
    finally:
        sk.skim_set_build_params(None)


def test_pull_on_degenerate_graphs(oracle_lib, restore_params):
    # every level pulled on a graph without edges, on p = 1 (every edge live
    # in every instance, so whole reach sets are searched) and with l = 1
    import paper_1408_6282_amd as sk
    sk.skim_set_build_params(dict(pull_frontier=1))
    rng = np.random.default_rng(12)
    src, dst, _ = random_small_graph(rng, 60, 240, [0xFFFFFFFF])
    cases = [(from_edges(40, [], []), 16, 8), (from_edges(60, src, dst, 0xFFFFFFFF), 64, 16),
             (from_edges(60, src, dst, 0xFFFFFFFF), 1, 4)]
    for g, ell, k in cases:
        log(f"pull: n={g.n} m={g.m} l={ell} k={k}")
        R, S, E, _, _ = gpu_build(g, ell, k, 7)
        R0, S0, _ = oracle_lib.build_alg2(g, 7, ell, k)
        assert np.array_equal(R, R0) and np.array_equal(S, S0)
