"""Resident sketches (skim_sketches_*): the handle keeps its own copy of the
sketch table and answers union queries with an enqueue-only launch.

* a handle built by skim_build_sketches_resident holds exactly the oracle's
  sketches, sizes and estimates;
* its queries equal skim_query_batch's results bit for bit (both
  estimators), and so do those of a handle copied from caller tables, after
  the caller's tables are overwritten;
* the query call captured into a HIP graph (torch.cuda.graph) and replayed
  several times, with eager work and synchronisations between replays and
  the sets rewritten in place, gives the eager results every time;
* offsets past nnodes or out of order give status -3 for that set only.
"""
import numpy as np
import pytest

from workloads import lognormal_query_sets
from workloads.configs import make_config, make_graph
from gpu_util import dev, gpu_build, gpu_query, log, to_dev_u32, to_dev_u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    cfg = make_config("tiny-ic")
    return cfg, make_graph(cfg)


def test_resident_build_equals_oracle(oracle_lib, tiny):
    import torch
    import paper_1408_6282_amd as sk
    cfg, g = tiny
    h = sk.Sketches.build(sk.DeviceGraph.from_host(g, dev()), cfg["ell"], cfg["k"], cfg["seed"])
    try:
        R, S, E = h.tables(torch)
    finally:
        h.free()
    R0, S0, _ = oracle_lib.build_alg2(g, cfg["seed"], cfg["ell"], cfg["k"])
    assert np.array_equal(R, R0) and np.array_equal(S, S0)
    assert np.array_equal(E, oracle_lib.estimates(R0, S0, cfg["k"], cfg["ell"]))


@pytest.mark.parametrize("estimator", [0, 1])
def test_resident_queries_equal_batch_call(tiny, estimator):
    import torch
    import paper_1408_6282_amd as sk
    cfg, g = tiny
    n, ell, k = g.n, cfg["ell"], cfg["k"]
    _, _, _, _, (rt, st) = gpu_build(g, ell, k, cfg["seed"])
    off, nodes = lognormal_query_sets(20000, n, 9)
    want, wst = gpu_query(rt, st, n, k, ell, off, nodes, estimator)
    h = sk.Sketches.from_tables(rt, st, n, k, ell)
    try:
        rt.fill_(0)  # the handle holds its own copy
        st.fill_(0)
        qo, qn = to_dev_u64(off), to_dev_u32(nodes)
        est = torch.empty(off.size - 1, dtype=torch.float64, device=dev())
        status = torch.empty(off.size - 1, dtype=torch.int32, device=dev())
        h.query(qo, qn, est, status, estimator=estimator)
        torch.cuda.synchronize()
        assert np.array_equal(est.cpu().numpy(), want)
        assert np.array_equal(status.cpu().numpy(), wst)
    finally:
        h.free()


def test_resident_query_captured_in_a_graph(tiny):
    import torch
    import paper_1408_6282_amd as sk
    cfg, g = tiny
    n, ell, k = g.n, cfg["ell"], cfg["k"]
    h = sk.Sketches.build(sk.DeviceGraph.from_host(g, dev()), ell, k, cfg["seed"])
    _, _, _, _, (rt, st) = gpu_build(g, ell, k, cfg["seed"])
    try:
        batches = [lognormal_query_sets(5000, n, 40 + j) for j in range(3)]
        cap = max(b[1].size for b in batches)
        qo = torch.zeros(5001, dtype=torch.int64, device=dev())
        qn = torch.zeros(cap, dtype=torch.int32, device=dev())
        est = torch.empty(5000, dtype=torch.float64, device=dev())
        status = torch.empty(5000, dtype=torch.int32, device=dev())
        ws = torch.zeros(16, dtype=torch.int64, device=dev())  # the graph's own counter

        def load(j):
            off, nodes = batches[j]
            qo.copy_(to_dev_u64(off))
            qn[:nodes.size].copy_(to_dev_u32(nodes))

        load(0)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):  # warm-up outside the capture
            h.query(qo, qn, est, status, workspace=ws, stream=s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            h.query(qo, qn, est, status, workspace=ws)
        for rep in range(6):
            j = rep % 3
            load(j)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            off, nodes = batches[j]
            want, wst = gpu_query(rt, st, n, k, ell, off, nodes, 0)  # eager work between replays
            assert np.array_equal(est.cpu().numpy(), want), f"replay {rep}"
            assert np.array_equal(status.cpu().numpy(), wst), f"replay {rep}"
        log("6 graph replays equal the batch call")
    finally:
        h.free()


def test_resident_query_bounds_offsets_on_the_device(tiny):
    import torch
    import paper_1408_6282_amd as sk
    cfg, g = tiny
    n, ell, k = g.n, cfg["ell"], cfg["k"]
    h = sk.Sketches.build(sk.DeviceGraph.from_host(g, dev()), ell, k, cfg["seed"])
    try:
        off = np.array([0, 2, 1, 4, 9], dtype=np.uint64)  # set 1 out of order; set 3 past nnodes
        nodes = np.array([1, 2, 3, 4, 5, 6], dtype=np.uint32)
        est = torch.empty(4, dtype=torch.float64, device=dev())
        status = torch.empty(4, dtype=torch.int32, device=dev())
        h.query(to_dev_u64(off), to_dev_u32(nodes), est, status)
        torch.cuda.synchronize()
        st = status.cpu().numpy()
        assert st[0] == 0 and st[1] == -3 and st[3] == -3
        assert est.cpu().numpy()[1] == 0.0 and est.cpu().numpy()[3] == 0.0
        with pytest.raises(sk.SkimError):
            h.query(to_dev_u64(off), to_dev_u32(nodes), est, status, estimator=2)
    finally:
        h.free()
