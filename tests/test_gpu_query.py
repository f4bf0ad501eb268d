"""GPU parity of skim_query_batch against the oracle: bottom-k and Cohen-Kaplan
estimators, batched and one-launch-per-query paths (identical bits), set
semantics, per-query status, and a sample of the batched lognormal workload."""
import numpy as np
import pytest

from workloads import from_edges, lognormal_query_sets, uniform_query_sets
from workloads.configs import make_config, make_graph
from brute import random_small_graph
from gpu_util import gpu_build, gpu_query, log

pytestmark = pytest.mark.gpu


def _sets(sets):
    off = np.zeros(len(sets) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(s) for s in sets])
    nodes = np.array([x for s in sets for x in s], dtype=np.uint32)
    return off, nodes


@pytest.fixture(scope="module")
def tiny(oracle_lib):
    cfg = make_config("tiny-ic")
    g = make_graph(cfg)
    R, S, E, _, (rt, st) = gpu_build(g, cfg["ell"], cfg["k"], cfg["seed"])
    return cfg, g, R, S, rt, st


def test_single_node_queries(oracle_lib, tiny):
    cfg, g, R, S, rt, st = tiny
    off = np.arange(g.n + 1, dtype=np.uint64)
    nodes = np.arange(g.n, dtype=np.uint32)
    for estimator, fn in [(0, oracle_lib.union_query), (1, oracle_lib.ck_query)]:
        want, _ = fn(R, S, cfg["k"], cfg["ell"], off, nodes)
        got, status = gpu_query(rt, st, g.n, cfg["k"], cfg["ell"], off, nodes, estimator)
        assert np.array_equal(got, want) and (status == 0).all()


@pytest.mark.parametrize("estimator", [0, 1])
def test_random_sets_batched_and_plain(oracle_lib, tiny, estimator):
    cfg, g, R, S, rt, st = tiny
    off, nodes = uniform_query_sets(600, g.n, 17, 1, 512)
    fn = oracle_lib.union_query if estimator == 0 else oracle_lib.ck_query
    want, _ = fn(R, S, cfg["k"], cfg["ell"], off, nodes)
    got, status = gpu_query(rt, st, g.n, cfg["k"], cfg["ell"], off, nodes, estimator, mode=0)
    plain, _ = gpu_query(rt, st, g.n, cfg["k"], cfg["ell"], off, nodes, estimator, mode=1)
    assert (status == 0).all()
    assert np.array_equal(got, want)
    assert np.array_equal(plain, got)


def test_set_semantics_and_status(oracle_lib, tiny):
    cfg, g, R, S, rt, st = tiny
    sets = [[], [3, 3, 3], [3], [1, 5000], [2, 0], list(range(1000)), [999, 0, 999]]
    off, nodes = _sets(sets)
    for estimator in (0, 1):
        got, status = gpu_query(rt, st, g.n, cfg["k"], cfg["ell"], off, nodes, estimator)
        assert got[0] == 0.0 and status[0] == 0
        assert got[1] == got[2]
        assert status[3] == -1 and got[3] == 0.0
        assert (status[[0, 1, 2, 4, 5, 6]] == 0).all()
        fn = oracle_lib.union_query if estimator == 0 else oracle_lib.ck_query
        want, wst = fn(R, S, cfg["k"], cfg["ell"], off, nodes)
        assert np.array_equal(got, want) and np.array_equal(status, wst)


def test_lognormal_batch_sample(oracle_lib, tiny):
    cfg, g, R, S, rt, st = tiny
    off, nodes = lognormal_query_sets(50_000, g.n, 104)
    want, _ = oracle_lib.union_query(R, S, cfg["k"], cfg["ell"], off, nodes)
    got, status = gpu_query(rt, st, g.n, cfg["k"], cfg["ell"], off, nodes, 0)
    assert (status == 0).all() and np.array_equal(got, want)


def test_random_graph_sketch_shapes(oracle_lib):
    rng = np.random.default_rng(9)
    for ell, k in [(1, 2), (64, 64), (8, 200)]:
        src, dst, thr = random_small_graph(rng, 50, 150, [0xFFFFFFFF // 3, 0xFFFFFFFF])
        g = from_edges(50, src, dst, thr)
        R, S, _, _, (rt, st) = gpu_build(g, ell, k, 3)
        off, nodes = uniform_query_sets(200, 50, 5, 1, 50)
        for estimator, fn in [(0, oracle_lib.union_query), (1, oracle_lib.ck_query)]:
            want, _ = fn(R, S, k, ell, off, nodes)
            got, _ = gpu_query(rt, st, 50, k, ell, off, nodes, estimator)
            log(f"ell={ell} k={k} est={estimator}")
            assert np.array_equal(got, want)


def test_bad_offsets_rejected(tiny):
    import paper_1408_6282_amd as sk
    cfg, g, R, S, rt, st = tiny
    off = np.array([0, 5, 3], dtype=np.uint64)
    nodes = np.arange(5, dtype=np.uint32)
    with pytest.raises(sk.SkimError) as ei:
        gpu_query(rt, st, g.n, cfg["k"], cfg["ell"], off, nodes)
    assert ei.value.status == sk.SKIM_EINVAL


def test_graph_plan_replays_match_batches(oracle_lib, tiny):
    """A captured plan, replayed several times with eager work and
    synchronisations in between, equals the batch call every time; sets
    rewritten in place are answered as rewritten; out-of-order offsets get
    status -3 without touching the sets that do not share them."""
    import torch
    import paper_1408_6282_amd as sk
    from gpu_util import to_dev_u64, to_dev_u32
    cfg, g, R, S, rt, st = tiny
    k, ell = cfg["k"], cfg["ell"]
    off, nodes = uniform_query_sets(500, g.n, 23, 1, 300)
    qo, qn = to_dev_u64(off), to_dev_u32(nodes)
    q = len(off) - 1
    for estimator, fn in [(0, oracle_lib.union_query), (1, oracle_lib.ck_query)]:
        est = torch.empty(q, dtype=torch.float64, device="cuda:0")
        status = torch.empty(q, dtype=torch.int32, device="cuda:0")
        plan = sk.QueryPlan(rt, st, g.n, k, ell, qo, qn, est, status, estimator=estimator)
        want, _ = fn(R, S, k, ell, off, nodes)
        for rep in range(4):
            est.fill_(-1.0)
            plan.launch()
            torch.cuda.synchronize()
            assert np.array_equal(est.cpu().numpy(), want), f"replay {rep}"
            assert (status.cpu().numpy() == 0).all()
            x = torch.arange(1 << 16, device="cuda:0").sum()  # eager work between replays
            torch.cuda.synchronize()
            assert int(x) == (1 << 16) * ((1 << 16) - 1) // 2
        # rewrite the sets in place (same offsets, other nodes)
        rng = np.random.default_rng(estimator)
        nodes2 = nodes.copy()
        for j in range(q):
            a, b = int(off[j]), int(off[j + 1])
            nodes2[a:b] = rng.choice(g.n, b - a, replace=False)
        qn.copy_(to_dev_u32(nodes2))
        plan.launch()
        torch.cuda.synchronize()
        want2, _ = fn(R, S, k, ell, off, nodes2)
        assert np.array_equal(est.cpu().numpy(), want2)
        # break the order of one offset in place
        bad = off.copy()
        bad[7] = bad[8] + 1
        qo.copy_(to_dev_u64(bad))
        plan.launch()
        torch.cuda.synchronize()
        stat = status.cpu().numpy()
        got = est.cpu().numpy()
        assert stat[7] == -3 and got[7] == 0.0  # its end now lies before its start
        # set 6 ends at the moved offset: a valid, longer set
        s6 = nodes2[int(off[6]):int(bad[7])]
        w6, _ = fn(R, S, k, ell, np.array([0, s6.size], dtype=np.uint64), s6)
        assert stat[6] == 0 and got[6] == w6[0]
        good = np.ones(q, dtype=bool)
        good[[6, 7]] = False
        assert (stat[good] == 0).all()
        assert np.array_equal(got[good], want2[good])
        qo.copy_(to_dev_u64(off))
        qn.copy_(to_dev_u32(nodes))
        plan.free()
