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


def test_failed_batch_completes_with_status_and_frees_its_slot(served):
    # The host-side hook makes the serving loop treat the next batch copy as
    # failed (nothing goes wrong on the device): that batch's requests
    # complete with -5, the slot serves the next batch normally, and the
    # server shuts down.
    import paper_1408_6282_amd as sk
    cfg, g, rt, st = served
    n, ell, k = g.n, cfg["ell"], cfg["k"]
    srv = sk.Server(rt, st, n, k, ell, budget_bytes=1 << 20, max_batch=64, streams=1)
    try:
        sk.skim_debug_inject(sk.SKIM_FAULT_SERVE, 1)
        t1 = srv.submit([1, 2, 3])
        r1 = _wait(lambda: srv.poll(t1))
        assert r1[1] == -5 and r1[0] == 0.0
        t2 = srv.submit([1, 2, 3])
        r2 = _wait(lambda: srv.poll(t2))
        want, _ = gpu_query(rt, st, n, k, ell, np.array([0, 3], dtype=np.uint64),
                            np.array([1, 2, 3], dtype=np.uint32))
        assert r2[1] == 0 and r2[0] == want[0]
    finally:
        sk.skim_debug_inject(sk.SKIM_FAULT_SERVE, 0)
        t0 = time.time()
        srv.close()
        assert time.time() - t0 < 30


def test_cancelled_requests_complete_with_status(served):
    # One query per batch on one stream, so that later requests still wait
    # when they are cancelled (a finished request cannot be cancelled:
    # SKIM_EINVAL).  The latest requests are cancelled first.
    import paper_1408_6282_amd as sk
    cfg, g, rt, st = served
    n, ell, k = g.n, cfg["ell"], cfg["k"]
    nodes = np.arange(512) % n
    want, _ = gpu_query(rt, st, n, k, ell, np.array([0, 512], dtype=np.uint64),
                        nodes.astype(np.uint32))
    srv = sk.Server(rt, st, n, k, ell, budget_bytes=64 << 20, max_batch=1, streams=1)
    try:
        tickets = [srv.submit(nodes) for _ in range(2000)]
        cancelled = set()
        for t in reversed(tickets[::2]):
            try:
                srv.cancel(t)
                cancelled.add(t)
            except sk.SkimError as e:
                assert e.status == sk.SKIM_EINVAL  # already finished
        assert cancelled, "no request was still waiting"
        for t in tickets:
            r = _wait(lambda: srv.poll(t))
            if t in cancelled:
                assert r[1] == -6 and r[0] == 0.0
            else:
                assert r[1] == 0 and r[0] == want[0]
        with pytest.raises(sk.SkimError):
            srv.cancel(tickets[1])  # finished and retired
    finally:
        srv.close()


def test_skim_requests_are_admitted_by_budget(served):
    import paper_1408_6282_amd as sk
    cfg, g, rt, st = served
    n, ell, k = g.n, cfg["ell"], cfg["k"]
    srv = sk.Server(rt, st, n, k, ell, budget_bytes=4096, max_batch=8, streams=1)
    try:
        srv.set_graph(sk.DeviceGraph.from_host(g, "cuda:0"), ell, k, cfg["seed"])
        with pytest.raises(sk.SkimError) as ei:
            srv.submit_greedy(1000)  # 12 * 1000 + 64 bytes > the whole budget
        assert ei.value.status == sk.SKIM_EUNSUPPORTED
        t = srv.submit_greedy(20)
        seeds, gains, _ = _wait(lambda: srv.poll_greedy(t, 20))
    finally:
        srv.close()
    ws, wg, _, _ = gpu_greedy(g, ell, k, cfg["seed"], [20])
    assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)


def test_injected_allocation_failure(served):
    # The next device allocation fails on the host side: the build returns
    # SKIM_ENOMEM with its outputs untouched, and the following build works.
    import torch
    import paper_1408_6282_amd as sk
    cfg, g, rt, st = served
    G = sk.DeviceGraph.from_host(g, "cuda:0")
    ranks = torch.full((g.n * cfg["k"],), 7, dtype=torch.int64, device="cuda:0")
    size = torch.full((g.n,), 7, dtype=torch.int32, device="cuda:0")
    sk.skim_debug_inject(sk.SKIM_FAULT_ALLOC, 1)
    try:
        with pytest.raises(sk.SkimError) as ei:
            sk.skim_build_sketches(G, cfg["ell"], cfg["k"], cfg["seed"], ranks, size)
        assert ei.value.status == sk.SKIM_ENOMEM
    finally:
        sk.skim_debug_inject(sk.SKIM_FAULT_ALLOC, 0)
    torch.cuda.synchronize()
    assert (ranks.cpu() == 7).all() and (size.cpu() == 7).all()
    sk.skim_build_sketches(G, cfg["ell"], cfg["k"], cfg["seed"], ranks, size)
    torch.cuda.synchronize()
    assert torch.equal(ranks, rt) and torch.equal(size, st)
