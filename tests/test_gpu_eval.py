"""GPU parity of skim_influence_batch, the exact influence evaluator of the
quality harness (Section 2, eqs. (Inf) and (timedinf)), against the oracle's
forward search per instance: every count bit for bit.

* random graphs over l, with empty sets, duplicate members and invalid nodes;
* SKIM's seed prefixes on the instances SKIM used: the evaluator must
  reproduce the cumulative gains (Section 4.1.1), and on 512 fresh instances
  (8 other seeds) the oracle's counts;
* the Chung-Lu graph at full size (10^6 nodes, 1.6 10^7 edges, l = 64);
* argument errors.
"""
import numpy as np
import pytest

from workloads import from_edges
from workloads.configs import make_config, make_graph
from brute import random_small_graph
from gpu_util import dev, gpu_greedy, log, to_dev_u32, to_dev_u64

pytestmark = pytest.mark.gpu


def gpu_influence(g, ell, seed, sets, G=None, status=True):
    import torch
    import paper_1408_6282_amd as sk
    G = G or sk.DeviceGraph.from_host(g, dev())
    off = np.zeros(len(sets) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(s) for s in sets])
    nodes = np.concatenate([np.asarray(s, dtype=np.uint32) for s in sets]) if off[-1] else None
    q = len(sets)
    out = torch.full((max(q, 1),), -5, dtype=torch.int64, device=dev())
    st = torch.full((max(q, 1),), 7, dtype=torch.int32, device=dev()) if status else None
    sk.skim_influence_batch(G, ell, seed, to_dev_u64(off),
                            to_dev_u32(nodes) if nodes is not None else None, out, st)
    torch.cuda.synchronize()
    r = out.cpu().numpy().view(np.uint64)[:q]
    return (r, st.cpu().numpy()[:q]) if status else r


@pytest.mark.parametrize("ell", [1, 5, 64])
def test_random_graphs_and_sets(oracle_lib, ell):
    rng = np.random.default_rng(ell + 40)
    for trial in range(4):
        n = int(rng.integers(2, 120))
        src, dst, thr = random_small_graph(rng, n, int(rng.integers(0, 4 * n)),
                                           [0xFFFFFFFF, 0xFFFFFFFF // 3, 0xFFFFFFFF // 20])
        g = from_edges(n, src, dst, thr)
        seed = int(rng.integers(0, 2 ** 62))
        sets = [[]]
        for _ in range(60):
            sz = int(rng.integers(1, min(n, 12) + 1))
            sets.append(rng.integers(0, n, size=sz).tolist())  # duplicates allowed
        sets.append([0, 0, 0])
        sets.append([n - 1, n])  # invalid: node n
        log(f"influence ell={ell} n={n} m={g.m} q={len(sets)} seed={seed}")
        got, st = gpu_influence(g, ell, seed, sets)
        for j, S in enumerate(sets):
            if max(S, default=-1) >= n:
                assert st[j] == -1 and got[j] == 0
                continue
            assert st[j] == 0
            assert int(got[j]) == oracle_lib.influence(g, seed, ell, sorted(set(S))), (j, S)


def test_skim_prefixes_same_and_fresh_instances(oracle_lib):
    cfg = make_config("served-skim")
    g = make_graph(cfg)
    ell, k, seed = cfg["ell"], cfg["k"], cfg["seed"]
    seeds, gains, _, _ = gpu_greedy(g, ell, k, seed, [200])
    prefixes = [seeds[:j].tolist() for j in (1, 2, 5, 10, 50, 100, 200)]
    log("influence: SKIM prefixes on SKIM's own instances")
    got, st = gpu_influence(g, ell, seed, prefixes)
    assert np.all(st == 0)
    cum = np.cumsum(gains.astype(np.uint64))
    assert [int(x) for x in got] == [int(cum[len(p) - 1]) for p in prefixes]
    for fresh in range(1, 9):  # 8 x 64 = 512 fresh instances
        log(f"influence: SKIM prefixes on fresh instances, seed {seed + 1000 * fresh}")
        got = gpu_influence(g, 64, seed + 1000 * fresh, prefixes, status=False)
        want = [oracle_lib.influence(g, seed + 1000 * fresh, 64, p) for p in prefixes]
        assert [int(x) for x in got] == want


@pytest.mark.slow
def test_chung_lu_1m_sets(oracle_lib):
    cfg = make_config("chung-lu-1m")
    log("generating chung-lu-1m")
    g = make_graph(cfg)
    rng = np.random.default_rng(77)
    outdeg = np.diff(g.row_ptr.astype(np.int64))
    hubs = np.argsort(outdeg)[::-1][:64].tolist()
    sets = [rng.integers(0, g.n, size=sz).tolist() for sz in (1, 1, 8, 64, 1000)]
    sets += [hubs[:1], hubs[:16], hubs]
    log("gpu influence chung-lu-1m")
    got, st = gpu_influence(g, cfg["ell"], cfg["seed"], sets)
    assert np.all(st == 0)
    for j, S in enumerate(sets):
        want = oracle_lib.influence(g, cfg["seed"], cfg["ell"], sorted(set(S)))
        log(f"  set {j} |S|={len(S)}: {int(got[j])} vs {want}")
        assert int(got[j]) == want


def test_errors_and_empty_batches():
    import torch
    import paper_1408_6282_amd as sk
    g = from_edges(6, [0, 1, 2], [1, 2, 3])
    G = sk.DeviceGraph.from_host(g, dev())
    r = torch.empty(2, dtype=torch.int64, device=dev())
    nodes = to_dev_u32([0, 1])
    # every set empty: no node array needed
    got = gpu_influence(g, 4, 1, [[], []], G=G, status=False)
    assert got.tolist() == [0, 0]
    # q = 0
    sk.skim_influence_batch(G, 4, 1, to_dev_u64([0]), None, r)
    for off in ([1, 1, 2], [0, 2, 1]):  # qoff[0] != 0; decreasing
        with pytest.raises(sk.SkimError) as ei:
            sk.skim_influence_batch(G, 4, 1, to_dev_u64(off), nodes, r)
        assert ei.value.status == sk.SKIM_EINVAL
    for ell in (0, 65):
        with pytest.raises(sk.SkimError) as ei:
            sk.skim_influence_batch(G, ell, 1, to_dev_u64([0, 1, 2]), nodes, r)
        assert ei.value.status == sk.SKIM_EINVAL
    with pytest.raises(sk.SkimError) as ei:  # sets hold nodes but no node array
        sk.skim_influence_batch(G, 4, 1, to_dev_u64([0, 1, 2]), None, r)
    assert ei.value.status == sk.SKIM_EINVAL


def gpu_greedy_exact(g, ell, seed, s):
    import torch
    import paper_1408_6282_amd as sk
    G = sk.DeviceGraph.from_host(g, dev())
    a = torch.full((max(s, 1),), -1, dtype=torch.int32, device=dev())
    b = torch.full((max(s, 1),), -1, dtype=torch.int64, device=dev())
    sk.skim_greedy_exact(G, ell, seed, s, a, b)
    torch.cuda.synchronize()
    return a.cpu().numpy().view(np.uint32)[:s], b.cpu().numpy().view(np.uint64)[:s]


@pytest.mark.parametrize("ell", [1, 8, 64])
def test_greedy_exact_matches_oracle(oracle_lib, ell):
    # the oracle's SKIM with k above every |R_u| is exact greedy (pinned
    # against brute force): every seed from the exhaustion rule
    rng = np.random.default_rng(ell + 70)
    for trial in range(3):
        n = int(rng.integers(2, 60))
        src, dst, thr = random_small_graph(rng, n, int(rng.integers(0, 3 * n)),
                                           [0xFFFFFFFF, 0xFFFFFFFF // 2, 0xFFFFFFFF // 10])
        g = from_edges(n, src, dst, thr)
        seed = int(rng.integers(0, 2 ** 62))
        s = n if trial == 0 else int(rng.integers(1, n + 1))
        log(f"greedy exact ell={ell} n={n} m={g.m} s={s}")
        seeds, gains = gpu_greedy_exact(g, ell, seed, s)
        ws, wg, cnt = oracle_lib.skim(g, seed, ell, n * ell + 1, s)
        assert cnt["fallback"] == s
        assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)


def test_greedy_exact_served_config(oracle_lib):
    cfg = make_config("served-skim")
    g = make_graph(cfg)
    log("greedy exact served-skim 50 seeds")
    seeds, gains = gpu_greedy_exact(g, cfg["ell"], cfg["seed"], 50)
    ws, wg, _ = oracle_lib.skim(g, cfg["seed"], cfg["ell"], g.n * cfg["ell"] + 1, 50)
    assert np.array_equal(seeds, ws) and np.array_equal(gains, wg)
    # the prefixes' influence on the same instances is the running sum of gains
    got = gpu_influence(g, cfg["ell"], cfg["seed"], [seeds[:j].tolist() for j in (1, 10, 50)],
                        status=False)
    cum = np.cumsum(gains)
    assert [int(v) for v in got] == [int(cum[0]), int(cum[9]), int(cum[49])]
