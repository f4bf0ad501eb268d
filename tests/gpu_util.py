"""Helpers for the GPU parity tests: run the HIP library on host data, return numpy."""
import sys

import numpy as np


def dev():
    import torch
    return torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_build(g, ell, k, seed, want_est=True):
    import torch
    import paper_1408_6282_amd as sk
    d = dev()
    G = sk.DeviceGraph.from_host(g, d)
    ranks = torch.empty(g.n * k, dtype=torch.int64, device=d)
    size = torch.empty(g.n, dtype=torch.int32, device=d)
    est = torch.empty(g.n, dtype=torch.float64, device=d) if want_est else None
    work = sk.skim_build_sketches(G, ell, k, seed, ranks, size, est)
    torch.cuda.synchronize()
    R = ranks.cpu().numpy().view(np.uint64).reshape(g.n, k)
    S = size.cpu().numpy().view(np.uint32)
    E = est.cpu().numpy() if want_est else None
    return R, S, E, work, (ranks, size)


def to_dev_u64(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(dev())


def to_dev_u32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(dev())


def gpu_query(ranks_t, size_t, n, k, ell, off, nodes, estimator=0, mode=0):
    import torch
    import paper_1408_6282_amd as sk
    qo = to_dev_u64(off)
    qn = to_dev_u32(nodes) if len(nodes) else torch.empty(0, dtype=torch.int32, device=dev())
    q = len(off) - 1
    est = torch.empty(max(q, 1), dtype=torch.float64, device=dev())
    st = torch.empty(max(q, 1), dtype=torch.int32, device=dev())
    sk.skim_query_batch(ranks_t, size_t, n, k, ell, qo, qn, est[:q] if q else est, st,
                        estimator=estimator, mode=mode)
    torch.cuda.synchronize()
    return est.cpu().numpy()[:q], st.cpu().numpy()[:q]


def gpu_greedy(g, ell, k, seed, chunks, G=None, records=False):
    """Run SKIM in the given chunk sizes with one resumed state; concatenated
    outputs (plus the per-seed tau and second largest sketch with records)."""
    import torch
    import paper_1408_6282_amd as sk
    d = dev()
    G = G or sk.DeviceGraph.from_host(g, d)
    state = sk.GreedyState()
    seeds, gains, gd = [], [], []
    try:
        for s in chunks:
            a = torch.empty(max(s, 1), dtype=torch.int32, device=d)
            b = torch.empty(max(s, 1), dtype=torch.int64, device=d)
            c = torch.empty(max(s, 1), dtype=torch.float64, device=d)
            sk.skim_greedy(G, ell, k, seed, s, a, b, c, state=state)
            torch.cuda.synchronize()
            seeds.append(a.cpu().numpy().view(np.uint32)[:s])
            gains.append(b.cpu().numpy().view(np.uint64)[:s])
            gd.append(c.cpu().numpy()[:s])
        sel = state.selected
        if records:
            tau = torch.empty(max(sel, 1), dtype=torch.int64, device=d)
            sec = torch.empty(max(sel, 1), dtype=torch.int32, device=d)
            sk.skim_greedy_records(state, 0, sel, tau, sec)
            torch.cuda.synchronize()
            rec = (tau.cpu().numpy().view(np.uint64)[:sel], sec.cpu().numpy().view(np.uint32)[:sel])
    finally:
        state.free()
    out = (np.concatenate(seeds), np.concatenate(gains), np.concatenate(gd), sel)
    return out + rec if records else out


def sha256(a) -> str:
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8)).hexdigest()


def golden(tag):
    """The oracle's stored counters and result digests (tests/golden/<tag>_counters.json,
    written by tests/golden/make_counters.py from the oracle alone)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        f"{tag}_counters.json")
    with open(path) as f:
        return json.load(f)


def check_digests(gold, g, R, S, E):
    """The GPU's sketches, sizes and estimates equal the oracle's, by digest."""
    from workloads.configs import graph_sha256
    assert gold["graph_sha256"] == graph_sha256(g), "stored digests are for another graph"
    d = gold["digests"]
    assert sha256(S.astype(np.uint32)) == d["size_sha256"], "sizes differ from the oracle's"
    assert sha256(R.astype(np.uint64)) == d["ranks_sha256"], "sketches differ from the oracle's"
    if E is not None:
        assert sha256(E.astype(np.float64)) == d["est_sha256"], "estimates differ from the oracle's"
