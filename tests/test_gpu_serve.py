"""GPU tests of the serving loop: every served result equals the batch call's
result for the same set (alone and in a mix with concurrent SKIM requests),
memory-budget admission refuses what does not fit, and SKIM through the server
equals the direct one-shot run."""
import time

import numpy as np
import pytest

from workloads import uniform_query_sets, poisson_arrivals
from workloads.configs import make_config, make_graph
from gpu_util import gpu_build, gpu_greedy, gpu_query, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    cfg = make_config("served-skim")
    g = make_graph(cfg)
    R, S, _, _, (rt, st) = gpu_build(g, cfg["ell"], cfg["k"], cfg["seed"])
    return cfg, g, rt, st


def _wait(fn, timeout=60.0):
    t = time.time()
    while True:
        r = fn()
        if r is not None:
            return r
        assert time.time() - t < timeout, "request did not complete"
        time.sleep(0.0005)


def test_served_queries_equal_batch_results_in_a_mix(served):
    import paper_1408_6282_amd as sk
    cfg, g, rt, st = served
    n, ell, k = g.n, cfg["ell"], cfg["k"]
    off, nodes = uniform_query_sets(3000, n, 77, 1, 512)
    want, wst = gpu_query(rt, st, n, k, ell, off, nodes, 0)
    srv = sk.Server(rt, st, n, k, ell, budget_bytes=8 << 20, max_batch=256, streams=4)
    try:
        srv.set_graph(sk.DeviceGraph.from_host(g, "cuda:0"), ell, k, cfg["seed"])
        gt = [srv.submit_greedy(50)]
        arr = poisson_arrivals(50_000.0, 3000 / 50_000.0, 5)[:3000]
        arr = np.concatenate([arr, np.full(3000 - arr.size, arr[-1] if arr.size else 0.0)])
        gt.append(srv.submit_greedy(50))
        est, status, lat, retries = srv.replay(off, nodes, arr)
        log(f"served 3000 queries: p50 {np.median(lat):.1f} us p99 {np.percentile(lat, 99):.1f} us "
            f"retries {retries}")
        assert np.array_equal(est, want) and np.array_equal(status, wst)
        seeds, gains = [], []
        for t in gt:
            a, b, _ = _wait(lambda: srv.poll_greedy(t, 50))
            seeds.append(a)
            gains.append(b)
    finally:
        srv.close()
    ws, wg, _, _ = gpu_greedy(g, ell, k, cfg["seed"], [100])
    assert np.array_equal(np.concatenate(seeds), ws) and np.array_equal(np.concatenate(gains), wg)


def test_submit_poll_and_admission(served):
    import paper_1408_6282_amd as sk
    cfg, g, rt, st = served
    n, ell, k = g.n, cfg["ell"], cfg["k"]
    srv = sk.Server(rt, st, n, k, ell, budget_bytes=4096, max_batch=8, streams=1)
    try:
        with pytest.raises(sk.SkimError) as ei:
            srv.submit(np.arange(1100) % 1000)  # 4 * 1100 + 20 bytes > the whole budget
        assert ei.value.status == sk.SKIM_EUNSUPPORTED
        t1 = srv.submit([1, 2, 3])
        t2 = srv.submit([5000])  # bad id: status -1 for this query only
        r1 = _wait(lambda: srv.poll(t1))
        r2 = _wait(lambda: srv.poll(t2))
        off = np.array([0, 3], dtype=np.uint64)
        want, _ = gpu_query(rt, st, n, k, ell, off, np.array([1, 2, 3], dtype=np.uint32))
        assert r1[0] == want[0] and r1[1] == 0
        assert r2[1] == -1
        with pytest.raises(sk.SkimError):
            srv.poll(t1)  # retired ticket
    finally:
        srv.close()
