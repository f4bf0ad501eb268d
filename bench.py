#!/usr/bin/env python
"""Benchmark of the sketch-based influence hot path on one MI355X.

A step is one combined-sketch build (live lists, rank windows, pruned
reverse searches, bottom-k merge, per-node estimates) of the 1M-node
Chung-Lu weighted-cascade workload (l = 64, k = 64) whose inputs are already
resident in HBM.  `value` is live-edge traversals per second, the numerator
being the oracle's exact count W_live for that workload (Algorithm 2's
work), not the kernels' own counts.

Beside it the same JSON line reports the roofline of the dominant kernel
(timed live with HIP events), the CPU oracle on a bounded sample, batched vs
one-launch-per-query throughput on the lognormal query workload, SKIM on
the served-SKIM configuration, and served-query latency.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "live-edge traversals/s (sketch build); batched vs plain queries/s, p99 latency"
# The dominant work: the pruned reverse searches, run by three kernels (the
# seed level of each window, whole-grid levels, and the workgroup tails);
# they are timed and counted together.
SEARCH_KERNELS = ["k_seed_window", "k_expand", "k_tails"]
DOMINANT = "search"
# Sources of the dominant kernel: measured HBM traffic is reported only while
# these are unchanged since the counters were taken.
DOMINANT_SOURCES = ["paper_1408_6282_amd/csrc/skim_build.hip",
                    "paper_1408_6282_amd/csrc/skim_internal.h"]
CALIBRATION_BYTES = 1 << 30
# Launch shapes of the R-MAT scale-24 build, chosen by a sweep over window
# spans, level batches and thread-per-entry limits on that graph.
RMAT_PARAMS = {"window_span": 3, "large_batch": 4, "thread_frontier": 2097152, "pull_frontier": 0}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def graph_digest(g):
    import hashlib
    h = hashlib.sha256()
    for a in (g.row_ptr, g.col, g.thr):
        h.update(memoryview(a).cast("B"))
    return h.hexdigest()


def oracle_counters(name, g, cfg):
    """The oracle's Algorithm-2 counters for this exact graph (stored, else computed)."""
    path = os.path.join(ROOT, "tests", "golden", f"{name.replace('-', '_')}_counters.json")
    dig = graph_digest(g)
    if os.path.exists(path):
        with open(path) as f:
            d = json.load(f)
        if (d["graph_sha256"] == dig and d["ell"] == cfg["ell"] and d["k"] == cfg["k"]
                and d["seed"] == cfg["seed"]):
            return d["counters"]
    log("stored oracle counters do not match this graph; running the oracle")
    import oracle
    _, _, cnt = oracle.build_alg2(g, cfg["seed"], cfg["ell"], cfg["k"])
    return cnt


def dominant_source_digest():
    import hashlib
    h = hashlib.sha256()
    for p in DOMINANT_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per build of the dominant kernel from the committed
    rocprofv3 PMC summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated, summed
    over its launches in one build), or None when the summary is missing or
    was taken on other kernel sources.  (Launches per build depend on the
    launch shapes the tuner picks; the bytes per build do not.)"""
    path = os.path.join(ROOT, "profiles", f"{DOMINANT}_{workload.replace('-', '_')}_traffic.txt")
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                key, val = line.split(":", 1)
                d[key.strip()] = val.strip()
    if d.get("kernel_source_sha256") != dominant_source_digest() or \
            "traffic_bytes_per_build" not in d:
        return None
    return float(d["traffic_bytes_per_build"])


def calibrate_copy():
    """A plain copy of known size (read and write CALIBRATION_BYTES each), run
    under rocprofv3 --pmc to scale FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    a = torch.ones(CALIBRATION_BYTES // 4, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.add(a, 1, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "int32 add, out of place", "read_bytes": CALIBRATION_BYTES,
                      "write_bytes": CALIBRATION_BYTES, "launches": 3}), flush=True)


def random_access_rates(torch, table_log2=27, n_log2=26, reps=3):
    """Random-access rates of this GPU, measured with plain library kernels on
    a 1 GiB table (far beyond the caches): 8-byte gathers (index_select) and
    8-byte atomic adds (index_add_ on int64) at 2^26 uniform random indices.
    The search's random accesses are of this kind: a 16-byte pair record read
    per live-edge scan, one CAS per accepted visit."""
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    table = torch.zeros(1 << table_log2, dtype=torch.int64, device=dev)
    idx = torch.randint(0, 1 << table_log2, (1 << n_log2,), device=dev, generator=gen)
    out = torch.empty(1 << n_log2, dtype=torch.int64, device=dev)
    ones = torch.ones_like(out)

    def rate(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return reps * (1 << n_log2) / (a.elapsed_time(b) / 1e3)

    gather = rate(lambda: torch.index_select(table, 0, idx, out=out))
    atomic = rate(lambda: table.index_add_(0, idx, ones))
    del table, idx, out, ones
    torch.cuda.empty_cache()
    return {"table_bytes": 8 << table_log2, "accesses": 1 << n_log2,
            "gather_per_s": gather, "atomic_add_per_s": atomic}


def algorithmic_bytes_search(cnt):
    """HBM floor of the pruned reverse searches (the traversal terms of the
    build's floor): every CSR edge read under perfect instance packing
    (source id + threshold, 8 B, C_min of them) and the offsets and instance
    mask of every packed expansion (16 B, N_exp of them)."""
    return 8 * cnt["c_min"] + 16 * cnt["n_exp"]


def algorithmic_bytes_build(cnt, n, k):
    """HBM floor of a whole build: the search floor plus the sketches (8 B per
    entry, n * k) and the estimates (8 B per node)."""
    return algorithmic_bytes_search(cnt) + 8 * n * k + 8 * n


def visit_model_bytes(cnt):
    """Bytes this design's search touches per unit of work when every access
    is counted once: per rank insertion the frontier entry (16 B: pair and
    source, live-list word) written and read back, the claimed pair record
    (16 B) and the record (8 B); per live-edge traversal the live source id
    (4 B) and the visited pair record (16 B)."""
    return cnt["n_ins"] * (16 + 16 + 16 + 8) + cnt["w_live"] * (4 + 16)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads(max_threads=16):
    return max(1, min(max_threads, os.cpu_count() or 1))


def cpu_baseline(g, cfg, max_threads=16):
    """The oracle's Algorithm 2 on the same workload (all l instances, one
    instance per thread at a time), on at most 16 host threads."""
    import oracle
    cores = host_threads(max_threads)
    t = time.perf_counter()
    _, _, cnt = oracle.build_alg2(g, cfg["seed"], cfg["ell"], cfg["k"], threads=cores)
    dt = time.perf_counter() - t
    return {"value": cnt["w_live"] / dt, "unit": "live-edge traversals/s",
            "cores": min(cores, cfg["ell"]), "kind": "oracle", "seconds": round(dt, 3),
            "cpu": cpu_model(),
            "sample": f"the whole workload: Algorithm 2 over all {cfg['ell']} instances "
                      f"(k={cfg['k']}, seed {cfg['seed']}); W_live = {cnt['w_live']}"}


def oracle_times(max_threads=16):
    """The oracle on the query and SKIM workloads, timed on this host: the
    1M lognormal union queries of batched-query (split over the host threads;
    the C oracle releases the interpreter lock) and SKIM's 200 seeds on
    served-skim (one thread: Algorithm 1 is sequential)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    from workloads import lognormal_query_sets
    from workloads.configs import make_config, make_graph
    cores = host_threads(max_threads)
    out = {"cpu": cpu_model(), "threads": cores}
    cfg = make_config("batched-query")
    g = make_graph(cfg)
    R, S, _ = oracle.build_alg2(g, cfg["seed"], cfg["ell"], cfg["k"], threads=cores)
    off, nodes = lognormal_query_sets(cfg["Q"], g.n, cfg["qseed"])
    Q = cfg["Q"]
    cuts = np.linspace(0, Q, cores + 1).astype(np.int64)

    def part(j):
        a, b = cuts[j], cuts[j + 1]
        return oracle.union_query(R, S, cfg["k"], cfg["ell"], off[a:b + 1] - off[a],
                                  nodes[off[a]:off[b]])
    t = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(part, range(cores)))
    dt = time.perf_counter() - t
    out["batched_query"] = {"queries": Q, "seconds": round(dt, 3), "queries_per_s": Q / dt,
                            "threads": cores}
    c5 = make_config("served-skim")
    g5 = make_graph(c5)
    t = time.perf_counter()
    oracle.skim(g5, c5["seed"], c5["ell"], c5["k"], c5["s"])
    dt = time.perf_counter() - t
    out["served_skim"] = {"seeds": c5["s"], "seconds": round(dt, 3), "threads": 1}
    return out


def bench_rmat(torch, sk, steps=2):
    """The rmat-24 build (scale 24, trivalency, l = 64, k = 32): time per
    build, live-edge traversals/s from the oracle's W_live, the whole-build
    floor, parity of the timed output against the oracle's stored digests,
    and the oracle's own time as stored with its host and threads."""
    from workloads.configs import make_config, make_graph
    cfg = make_config("rmat-24")
    log("generating rmat-24")
    g = make_graph(cfg)
    gold = golden_record("rmat_24")
    if gold is None or gold["graph_sha256"] != graph_digest(g):
        return {"skipped": "no stored oracle result for this graph"}
    cnt = gold["counters"]
    dev = torch.device("cuda:0")
    G = sk.DeviceGraph.from_host(g, dev)
    n, ell, k, seed = g.n, cfg["ell"], cfg["k"], cfg["seed"]
    ranks = torch.empty(n * k, dtype=torch.int64, device=dev)
    size = torch.empty(n, dtype=torch.int32, device=dev)
    est = torch.empty(n, dtype=torch.float64, device=dev)
    # launch shapes for this graph (the tuner's choice for the 1M-node graph
    # is not carried over; a tuning pass here would cost minutes)
    saved = sk.skim_get_build_params()
    sk.skim_set_build_params(RMAT_PARAMS)
    try:
        log("rmat-24 warm-up build")
        work = sk.skim_build_sketches(G, ell, k, seed, ranks, size, est)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            work = sk.skim_build_sketches(G, ell, k, seed, ranks, size, est)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / steps
    finally:
        sk.skim_set_build_params(saved)
    log(f"rmat-24: {sec * 1e3:.1f} ms per build; {work}")
    floor = algorithmic_bytes_build(cnt, n, k)
    out = {"workload": "rmat-24", "n": n, "m": g.m, "ell": ell, "k": k, "steps": steps,
           "ms_per_build": sec * 1e3, "build_params": RMAT_PARAMS, "live_edge_traversals_per_s": cnt["w_live"] / sec,
           "oracle_counters": cnt, "device_work": work,
           "build_floor_bytes": floor, "build_floor_ms": floor / (HBM_PEAK_GBS * 1e9) * 1e3,
           "build_floor_over_measured": floor / (HBM_PEAK_GBS * 1e9) / sec,
           "parity": output_parity("rmat-24", g, cfg, ranks, size, est),
           "oracle_stored": {"seconds": gold.get("oracle_seconds"),
                             "threads": gold.get("oracle_threads"), "cpu": gold.get("oracle_cpu"),
                             "live_edge_traversals_per_s":
                                 cnt["w_live"] / gold["oracle_seconds"]
                                 if gold.get("oracle_seconds") else None}}
    del G, ranks, size, est
    torch.cuda.empty_cache()
    # the searches' random accesses at the rates plain gathers and atomics
    # reach on a table the size of this build's pair records (17 GB: no
    # cache holds it)
    try:
        ra = random_access_rates(torch, table_log2=31)
        floor_s = work["scans"] / ra["gather_per_s"] + work["visits"] / ra["atomic_add_per_s"]
        ra.update({"scans": work["scans"], "visits": work["visits"],
                   "search_floor_ms": floor_s * 1e3, "search_floor_over_build": floor_s / sec})
        out["random_access"] = ra
    except RuntimeError as e:  # not enough free device memory for the table
        out["random_access"] = {"skipped": str(e)[:200]}
        torch.cuda.empty_cache()
    return out


def golden_record(tag):
    path = os.path.join(ROOT, "tests", "golden", f"{tag}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def output_parity(tag, g, cfg, ranks, size, est):
    """The build's outputs against the oracle's stored result digests (SHA-256
    of the sketches, sizes and estimates that tests/golden/make_counters.py
    wrote from the oracle alone): True/False, or None when no digest matches
    this graph and configuration."""
    import hashlib
    d = golden_record(tag.replace("-", "_"))
    if (d is None or "digests" not in d or d["graph_sha256"] != graph_digest(g)
            or d["ell"] != cfg["ell"] or d["k"] != cfg["k"] or d["seed"] != cfg["seed"]):
        return None
    dig = lambda t: hashlib.sha256(t.cpu().numpy().view(np.uint8)).hexdigest()  # noqa: E731
    ok = dig(ranks) == d["digests"]["ranks_sha256"] and dig(size) == d["digests"]["size_sha256"]
    if est is not None:
        ok = ok and dig(est) == d["digests"]["est_sha256"]
    return bool(ok)


def bench_build(args, torch, sk, g, cfg):
    """Time K builds, then time the dominant kernel's launches with HIP events
    over another K builds.  The two passes are separate because recording two
    events around each of the kernel's ~500 launches per build slows the build
    itself (host work and stream markers), which would understate `value`."""
    dev = torch.device("cuda:0")
    G = sk.DeviceGraph.from_host(g, dev)
    n, ell, k, seed = g.n, cfg["ell"], cfg["k"], cfg["seed"]
    ranks = torch.empty(n * k, dtype=torch.int64, device=dev)
    size = torch.empty(n, dtype=torch.int32, device=dev)
    est = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    tuning = None
    if not args.no_tune:
        cache = args.tune_cache
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        best, best_ms, start_ms, hit = sk.skim_tune_build_cached(G, ell, k, seed, ranks, size,
                                                                 cache, reps=2, stream=stream)
        tuning = {"params": best, "best_ms": best_ms, "default_ms": start_ms, "cache_hit": hit,
                  "cache": cache}
        log(f"autotuned {tuning}")
    for w in range(args.warmup):
        work = sk.skim_build_sketches(G, ell, k, seed, ranks, size, est, stream=stream)
        log(f"warmup {w}: {work}")
    sk.skim_timing_enable(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        work = sk.skim_build_sketches(G, ell, k, seed, ranks, size, est, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"timed {args.steps} steps: {(t1 - t0) * 1e3 / args.steps:.3f} ms/step; {work}")
    parity = output_parity(args.workload, g, cfg, ranks, size, est)
    log(f"parity of the last timed build: {parity}")
    # kernel pass: every launch of the dominant kernel bracketed by HIP events
    # on the stream it is launched on
    sk.skim_timing_reset()
    sk.skim_timing_enable(",".join(SEARCH_KERNELS))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for s in range(args.steps):
        sk.skim_build_sketches(G, ell, k, seed, ranks, size, est, stream=stream)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    sk.skim_timing_enable(None)
    kms, klaunch, per_kernel = 0.0, 0, {}
    for name in SEARCH_KERNELS:
        ms_, n_ = sk.skim_timing_read(name)
        per_kernel[name] = {"ms_per_step": ms_ / args.steps, "launches_per_step": n_ / args.steps}
        kms += ms_
        klaunch += n_
    log(f"kernel pass {args.steps} steps: {(t3 - t2) * 1e3 / args.steps:.3f} ms/step")
    return (t1 - t0) / args.steps, work, kms, klaunch, (t3 - t2) / args.steps, tuning, parity, \
        per_kernel


def bench_queries(torch, sk, reps=5, plain_q=20000):
    from workloads import lognormal_query_sets
    from workloads.configs import make_config, make_graph
    cfg = make_config("batched-query")
    g = make_graph(cfg)
    dev = torch.device("cuda:0")
    G = sk.DeviceGraph.from_host(g, dev)
    n, ell, k = g.n, cfg["ell"], cfg["k"]
    ranks = torch.empty(n * k, dtype=torch.int64, device=dev)
    size = torch.empty(n, dtype=torch.int32, device=dev)
    sk.skim_build_sketches(G, ell, k, cfg["seed"], ranks, size)
    off, nodes = lognormal_query_sets(cfg["Q"], n, cfg["qseed"])
    qo = torch.from_numpy(off.view(np.int64)).to(dev)
    qn = torch.from_numpy(nodes.view(np.int32)).to(dev)
    Q = cfg["Q"]
    est = torch.empty(Q, dtype=torch.float64, device=dev)
    sk.skim_query_batch(ranks, size, n, k, ell, qo, qn, est)  # warm-up
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        sk.skim_query_batch(ranks, size, n, k, ell, qo, qn, est)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    tb = float(np.median(times))
    # the same batch as a captured HIP graph, replayed
    gest = torch.empty(Q, dtype=torch.float64, device=dev)
    plan = sk.QueryPlan(ranks, size, n, k, ell, qo, qn, gest)
    plan.launch()
    torch.cuda.synchronize()
    gtimes = []
    for _ in range(reps):
        t = time.perf_counter()
        plan.launch()
        torch.cuda.synchronize()
        gtimes.append(time.perf_counter() - t)
    tg = float(np.median(gtimes))
    same_graph = bool(torch.equal(gest, est))
    plan.free()
    # plain path: one launch per query, on the first plain_q queries
    po = qo[:plain_q + 1].clone()
    pest = torch.empty(plain_q, dtype=torch.float64, device=dev)
    sk.skim_query_batch(ranks, size, n, k, ell, po, qn, pest, mode=1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sk.skim_query_batch(ranks, size, n, k, ell, po, qn, pest, mode=1)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    same = bool(torch.equal(pest, est[:plain_q]))
    sizes = np.diff(off.astype(np.int64))
    return {"workload": "batched-query", "queries": Q, "mean_set_size": round(float(sizes.mean()), 3),
            "batched_queries_per_s": Q / tb, "batched_ms": tb * 1e3,
            "graph_queries_per_s": Q / tg, "graph_ms": tg * 1e3, "graph_identical": same_graph,
            "plain_queries_per_s": plain_q / tp, "plain_sample": plain_q,
            "batched_over_plain": (Q / tb) / (plain_q / tp), "identical_estimates": same}


def bench_skim(torch, sk, reps=3):
    from workloads.configs import make_config, make_graph
    cfg = make_config("served-skim")
    g = make_graph(cfg)
    dev = torch.device("cuda:0")
    G = sk.DeviceGraph.from_host(g, dev)
    s = cfg["s"]
    seeds = torch.empty(s, dtype=torch.int32, device=dev)
    gains = torch.empty(s, dtype=torch.int64, device=dev)
    sk.skim_greedy(G, cfg["ell"], cfg["k"], cfg["seed"], s, seeds, gains)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        sk.skim_greedy(G, cfg["ell"], cfg["k"], cfg["seed"], s, seeds, gains)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    t = float(np.median(times))
    out = {"workload": "served-skim", "seeds": s, "ms": t * 1e3, "seeds_per_s": s / t,
           "influence_pairs": int(gains.sum().item())}
    out["adaptive_error"] = bench_adaptive(torch, sk, G, cfg, s, reps)
    out["fresh_instances"] = bench_fresh(torch, sk, G, cfg, seeds, gains)
    out["vs_exact_greedy"] = bench_exact_greedy(torch, sk, G, cfg, gains)
    out["chung_lu_20k_wc"] = bench_skim_20k(torch, sk)
    return out


def bench_skim_20k(torch, sk, s=50):
    """SKIM on a heavy-tailed graph: Chung-Lu n = 20,000, m = 320,000, weighted
    cascade, l = k = 64, 50 seeds (one call, state built inside)."""
    from workloads.graphs import Graph, chung_lu_graph, wc_thresholds
    dev = torch.device("cuda:0")
    n = 20000
    rp, col = chung_lu_graph(n, 320000, 2.1, 56)
    g = Graph(n, rp, col, wc_thresholds(rp, col, n))
    G = sk.DeviceGraph.from_host(g, dev)
    seeds = torch.empty(s, dtype=torch.int32, device=dev)
    gains = torch.empty(s, dtype=torch.int64, device=dev)
    sk.skim_greedy(G, 64, 64, 1, s, seeds, gains)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sk.skim_greedy(G, 64, 64, 1, s, seeds, gains)
    torch.cuda.synchronize()
    t = time.perf_counter() - t
    return {"n": n, "m": g.m, "ell": 64, "k": 64, "seeds": s, "ms": t * 1e3,
            "influence": float(gains.sum().item()) / 64}


def bench_skim_1m(torch, sk, g, cfg, reps=3):
    """SKIM on the 1M-node weighted-cascade graph (l = k = 64), as many seeds
    as the oracle's stored run, one call with the state built inside; the
    sequence is compared with the oracle's and the oracle's single-thread time
    is reported beside it."""
    path = os.path.join(ROOT, "tests", "golden", "chung_lu_1m_skim.json")
    with open(path) as f:
        gold = json.load(f)
    from workloads.configs import graph_sha256
    if gold["graph_sha256"] != graph_sha256(g):
        return {"skipped": "stored oracle sequence is for another graph"}
    dev = torch.device("cuda:0")
    G = sk.DeviceGraph.from_host(g, dev)
    s = gold["s"]
    seeds = torch.empty(s, dtype=torch.int32, device=dev)
    gains = torch.empty(s, dtype=torch.int64, device=dev)
    times = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t = time.perf_counter()
        sk.skim_greedy(G, cfg["ell"], cfg["k"], cfg["seed"], s, seeds, gains)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    t = float(np.median(times[1:]))
    parity = (seeds.cpu().numpy().view(np.uint32).tolist() == gold["seeds"]
              and gains.cpu().numpy().view(np.uint64).tolist() == gold["gain_pairs"])
    return {"workload": "chung-lu-1m", "n": g.n, "m": g.m, "ell": cfg["ell"], "k": cfg["k"],
            "seeds": s, "ms": t * 1e3, "parity": parity,
            "influence": float(gains.sum().item()) / cfg["ell"],
            "oracle_seconds": gold["oracle_seconds"], "oracle_threads": gold["oracle_threads"],
            "oracle_cpu": gold["oracle_cpu"], "oracle_over_gpu": gold["oracle_seconds"] / t}


def bench_exact_greedy(torch, sk, G, cfg, skim_gains, s=50):
    """SKIM against exact greedy on the same 64 instances (Section 4's
    comparison): the influence of the first s seeds of each, and the time of
    the exact greedy that scores every node at every step."""
    dev = torch.device("cuda:0")
    seeds = torch.empty(s, dtype=torch.int32, device=dev)
    gains = torch.empty(s, dtype=torch.int64, device=dev)
    sk.skim_greedy_exact(G, cfg["ell"], cfg["seed"], s, seeds, gains)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sk.skim_greedy_exact(G, cfg["ell"], cfg["seed"], s, seeds, gains)
    torch.cuda.synchronize()
    t = time.perf_counter() - t
    ex = float(gains[:s].sum().item()) / cfg["ell"]
    sk_inf = float(skim_gains[:s].sum().item()) / cfg["ell"]
    return {"seeds": s, "exact_greedy_ms": t * 1e3, "exact_greedy_influence": ex,
            "skim_influence": sk_inf, "skim_over_exact": sk_inf / ex}


def bench_fresh(torch, sk, G, cfg, seeds, gains, groups=8):
    """Quality harness: the influence of every prefix of the SKIM seed sequence
    on 64 * groups fresh instances (seeds the sketches never used), by the
    exact evaluator, against SKIM's own in-sample gains."""
    dev = torch.device("cuda:0")
    ell = cfg["ell"]
    S = seeds.cpu().numpy().view(np.uint32)
    s = S.size
    off = np.zeros(s + 1, dtype=np.uint64)
    off[1:] = np.cumsum(np.arange(1, s + 1, dtype=np.uint64))
    nodes = np.concatenate([S[:j] for j in range(1, s + 1)])
    qo = torch.from_numpy(off.view(np.int64)).to(dev)
    qn = torch.from_numpy(nodes.view(np.int32)).to(dev)
    reach = torch.empty(s, dtype=torch.int64, device=dev)
    total = np.zeros(s)
    times, visits = [], 0
    for gix in range(groups):
        fresh_seed = cfg["seed"] + 7919 * (gix + 1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sk.skim_influence_batch(G, 64, fresh_seed, qo, qn, reach)
        times.append(time.perf_counter() - t)
        r = reach.cpu().numpy().view(np.uint64).astype(np.float64)
        total += r
        visits += int(r.sum())
    fresh = total / (64 * groups)
    insample = np.cumsum(gains.cpu().numpy().astype(np.float64)) / ell
    t = float(np.median(times))
    return {"instances": 64 * groups, "sets": s, "member_nodes": int(nodes.size),
            "ms_per_call": t * 1e3, "pair_visits_per_s": visits / groups / t,
            "influence_200_fresh": float(fresh[-1]), "influence_200_in_sample": float(insample[-1]),
            "influence_50_fresh": float(fresh[49]), "influence_50_in_sample": float(insample[49]),
            "max_rel_gap_prefixes": float(np.max(np.abs(fresh - insample) / fresh))}


def tail_convolution_flops(s, bins):
    """Multiply-adds of the pairwise tree of capped convolutions, 2 flops each:
    every pair of rows costs sum_{j=0..bins} (j + 1)."""
    per_pair = (bins + 1) * (bins + 2) // 2
    rows, pairs = s, 0
    while rows > 1:
        pairs += rows // 2
        rows = (rows + 1) // 2
    return 2 * pairs * per_pair


def bench_adaptive(torch, sk, G, cfg, s, reps, bins=4096, rel=0.25):
    """The adaptive error estimate of the same 200-seed run: records from a
    resumable state, then the confidence distribution of the total
    discrepancy (Section 4), timed per call."""
    dev = torch.device("cuda:0")
    state = sk.GreedyState()
    try:
        seeds = torch.empty(s, dtype=torch.int32, device=dev)
        gains = torch.empty(s, dtype=torch.int64, device=dev)
        sk.skim_greedy(G, cfg["ell"], cfg["k"], cfg["seed"], s, seeds, gains, state=state)
        tau = torch.empty(s, dtype=torch.int64, device=dev)
        second = torch.empty(s, dtype=torch.int32, device=dev)
        sk.skim_greedy_records(state, 0, s, tau, second)
    finally:
        state.free()
    tail = torch.empty(bins + 1, dtype=torch.float64, device=dev)
    sk.skim_discrepancy_tail(tau, second, gains, bins, rel, tail)
    times = []
    for _ in range(max(reps, 5)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        sk.skim_discrepancy_tail(tau, second, gains, bins, rel, tail)
        times.append(time.perf_counter() - t)
    t = float(np.median(times))
    T = tail.cpu().numpy()
    flops = tail_convolution_flops(s, bins)
    at = {f"{x:g}": float(T[int(round(x / rel * bins))]) for x in (0.01, 0.02, 0.05, 0.1, 0.25)}
    return {"bins": bins, "max_rel_error": rel, "ms": t * 1e3,
            "conv_tflops": flops / t / 1e12, "fp64_peak_tflops": 78.6,
            "filled_seeds": int((tau != -1).sum().item()),
            "p_total_discrepancy_at_least": at}


def bench_oracle_quality(torch, sk, g, cfg, sets_per_size=100):
    """The influence oracle's accuracy as the paper tabulates it (Section 6.2):
    seed sets of 1, 50 and 1000 nodes, drawn uniformly or by the neighbourhood
    generator; estimates from the sketches (bottom-k and Cohen-Kaplan) against
    the exact influence on the same l instances (skim_influence_batch)."""
    from workloads import neighbourhood_query_sets, uniform_query_sets
    dev = torch.device("cuda:0")
    ell, k, seed = cfg["ell"], cfg["k"], cfg["seed"]
    G = sk.DeviceGraph.from_host(g, dev)
    ranks = torch.empty(g.n * k, dtype=torch.int64, device=dev)
    size = torch.empty(g.n, dtype=torch.int32, device=dev)
    sk.skim_build_sketches(G, ell, k, seed, ranks, size)
    out = {}
    for s in (1, 50, 1000):
        gens = {"uniform": uniform_query_sets(sets_per_size, g.n, 500 + s, s, s),
                "neighbourhood": neighbourhood_query_sets(g.row_ptr, g.col, g.n, sets_per_size, s,
                                                          600 + s)}
        for name, (off, nodes) in gens.items():
            qo = torch.from_numpy(off.view(np.int64)).to(dev)
            qn = torch.from_numpy(nodes.view(np.int32)).to(dev)
            q = off.size - 1
            reach = torch.empty(q, dtype=torch.int64, device=dev)
            sk.skim_influence_batch(G, ell, seed, qo, qn, reach)
            exact = reach.cpu().numpy().astype(np.float64) / ell
            row = {"exact_mean": float(exact.mean())}
            for est_name, estimator in (("bottom_k", 0), ("cohen_kaplan", 1)):
                est = torch.empty(q, dtype=torch.float64, device=dev)
                sk.skim_query_batch(ranks, size, g.n, k, ell, qo, qn, est, estimator=estimator)
                torch.cuda.synchronize()
                t = time.perf_counter()
                sk.skim_query_batch(ranks, size, g.n, k, ell, qo, qn, est, estimator=estimator)
                torch.cuda.synchronize()
                t = time.perf_counter() - t
                e = est.cpu().numpy()
                row[est_name] = {"mean_rel_error_pct": float(np.mean(np.abs(e - exact) / exact)) * 100,
                                 "us_per_query_batched": t / q * 1e6}
            out[f"s{s}_{name}"] = row
    return out


def bench_error_vs_ell(torch, sk, groups=128, nodes=200, k=64):
    """Error against the IC model itself (Section 6.2's figure on l): the
    influence of sample nodes estimated from sketches built on l instances,
    and from the IC-model sketches, against their influence on 64 * groups
    fresh instances (exact evaluator), on a 20,000-node weighted-cascade
    Chung-Lu graph."""
    from workloads.graphs import Graph, chung_lu_graph, wc_thresholds
    dev = torch.device("cuda:0")
    n = 20000
    rp, col = chung_lu_graph(n, 320000, 2.1, 57)
    g = Graph(n, rp, col, wc_thresholds(rp, col, n))
    G = sk.DeviceGraph.from_host(g, dev)
    rng = np.random.default_rng(58)
    sample = np.sort(rng.choice(n, size=nodes, replace=False)).astype(np.uint32)
    off = np.arange(nodes + 1, dtype=np.uint64)
    qo = torch.from_numpy(off.view(np.int64)).to(dev)
    qn = torch.from_numpy(sample.view(np.int32)).to(dev)
    reach = torch.empty(nodes, dtype=torch.int64, device=dev)
    truth = np.zeros(nodes)
    t = time.perf_counter()
    for gi in range(groups):
        sk.skim_influence_batch(G, 64, 10_000 + gi, qo, qn, reach)
        truth += reach.cpu().numpy().astype(np.float64)
    t_truth = time.perf_counter() - t
    truth /= 64 * groups
    out = {"graph": "chung-lu-20k-wc", "sample_nodes": nodes, "k": k,
           "reference_instances": 64 * groups, "reference_ms": t_truth * 1e3}
    for ell in (1, 4, 16, 64):
        ranks = torch.empty(n * k, dtype=torch.int64, device=dev)
        size = torch.empty(n, dtype=torch.int32, device=dev)
        est = torch.empty(n, dtype=torch.float64, device=dev)
        sk.skim_build_sketches(G, ell, k, 1, ranks, size, est)
        e = est.cpu().numpy()[sample.astype(np.int64)]
        out[f"l{ell}_mean_rel_error_pct"] = float(np.mean(np.abs(e - truth) / truth)) * 100
    pos = torch.empty(n * k, dtype=torch.int32, device=dev)
    est = torch.empty(n, dtype=torch.float64, device=dev)
    sk.skim_build_ic_sketches(G, k, 1, pos, est)
    e = est.cpu().numpy()[sample.astype(np.int64)]
    out["ic_model_mean_rel_error_pct"] = float(np.mean(np.abs(e - truth) / truth)) * 100
    return out


def bench_ic(torch, sk, reps=3):
    """IC-model sketches (structured permutation ranks, Section 3) on served-skim
    and on a 20,000-node weighted-cascade Chung-Lu graph, k = 64."""
    from workloads.configs import make_config, make_graph
    from workloads.graphs import Graph, chung_lu_graph, wc_thresholds
    dev = torch.device("cuda:0")
    cfg = make_config("served-skim")
    rp, col = chung_lu_graph(20000, 320000, 2.1, 56)
    graphs = [("served-skim", make_graph(cfg)),
              ("chung-lu-20k-wc", Graph(20000, rp, col, wc_thresholds(rp, col, 20000)))]
    out = {}
    k = 64
    for name, g in graphs:
        G = sk.DeviceGraph.from_host(g, dev)
        pos = torch.empty(g.n * k, dtype=torch.int32, device=dev)
        est = torch.empty(g.n, dtype=torch.float64, device=dev)
        sk.skim_build_ic_sketches(G, k, cfg["seed"], pos, est)
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            sk.skim_build_ic_sketches(G, k, cfg["seed"], pos, est)
            times.append(time.perf_counter() - t)
        t = float(np.median(times))
        out[name] = {"n": g.n, "m": g.m, "k": k, "ms": t * 1e3,
                     "positions_per_s": g.n * k / t,
                     "mean_estimate": float(est.mean().item())}
        if name == "served-skim":
            out[name]["union_queries"] = bench_ic_queries(torch, sk, pos, g.n, k)
    return out


def bench_ic_queries(torch, sk, pos, n, k, Q=1_000_000):
    """Union queries over IC-model sketches: the lognormal batch of the
    batched-query workload (mean |S| about 12), both estimators."""
    from workloads import lognormal_query_sets
    dev = torch.device("cuda:0")
    off, nodes = lognormal_query_sets(Q, n, 3)
    qo = torch.from_numpy(off.view(np.int64)).to(dev)
    qn = torch.from_numpy(nodes.view(np.int32)).to(dev)
    est = torch.empty(Q, dtype=torch.float64, device=dev)
    out = {"queries": Q}
    for name, estimator in (("bottom_k", 0), ("cohen_kaplan", 1)):
        sk.skim_ic_query_batch(pos, n, k, qo, qn, est, estimator=estimator)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sk.skim_ic_query_batch(pos, n, k, qo, qn, est, estimator=estimator)
        torch.cuda.synchronize()
        out[f"{name}_queries_per_s"] = Q / (time.perf_counter() - t)
    return out


def bench_serving(torch, sk, duration=None, sweep_queries=300_000):
    """Served queries on the served-skim sketches (sets of U[1, 512] nodes):

    * the configured open-loop Poisson stream (50k queries/s for 10 s) with
      four incremental 50-seed SKIM requests overlapping on the device:
      p50/p99 latency and completed queries/s;
    * a capacity sweep: open-loop streams offered above the plain path's
      rate (0.5M/s and 2M/s) and every request at t = 0 (saturation),
      completed queries/s, p50/p99 and admission retries each;
    * the plain path (one launch per query) on the same kind of sets, so that
      served capacity is compared with it at identical estimates."""
    from workloads import uniform_query_sets, poisson_arrivals
    from workloads.configs import make_config, make_graph
    cfg = make_config("served-skim")
    duration = cfg["duration"] if duration is None else duration
    g = make_graph(cfg)
    dev = torch.device("cuda:0")
    G = sk.DeviceGraph.from_host(g, dev)
    n, ell, k = g.n, cfg["ell"], cfg["k"]
    ranks = torch.empty(n * k, dtype=torch.int64, device=dev)
    size = torch.empty(n, dtype=torch.int32, device=dev)
    sk.skim_build_sketches(G, ell, k, cfg["seed"], ranks, size)

    def reference(off, nodes):
        qo = torch.from_numpy(off.view(np.int64)).to(dev)
        qn = torch.from_numpy(nodes.view(np.int32)).to(dev)
        ref = torch.empty(off.size - 1, dtype=torch.float64, device=dev)
        sk.skim_query_batch(ranks, size, n, k, ell, qo, qn, ref)
        return ref.cpu().numpy()

    arr = poisson_arrivals(cfg["rate"], duration, cfg["qseed"])
    off, nodes = uniform_query_sets(arr.size, n, cfg["qseed"] + 1, 1, 512)
    srv = sk.Server(ranks, size, n, k, ell, budget_bytes=64 << 20, max_batch=4096, streams=4)
    try:
        srv.set_graph(G, ell, k, cfg["seed"])
        tickets = [srv.submit_greedy(50) for _ in range(cfg["s"] // 50)]
        t = time.perf_counter()
        est, status, lat, retries = srv.replay(off, nodes, arr)
        wall = time.perf_counter() - t
        greedy_lat = []
        for tk in tickets:
            while True:
                r = srv.poll_greedy(tk, 50)
                if r is not None:
                    greedy_lat.append(r[2])
                    break
                time.sleep(0.001)
    finally:
        srv.close()
    same = bool(np.array_equal(reference(off, nodes), est))
    out = {"workload": "served-skim", "rate_per_s": cfg["rate"], "duration_s": duration,
           "queries": int(arr.size), "completed_queries_per_s": arr.size / wall,
           "p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
           "admission_retries": retries, "skim_requests": len(tickets),
           "skim_request_latency_ms": [round(x / 1e3, 3) for x in greedy_lat],
           "identical_to_batch": same}
    del off, nodes, est, lat

    # the plain path on U[1, 512] sets: one launch per query
    poff, pnodes = uniform_query_sets(20_000, n, cfg["qseed"] + 2, 1, 512)
    qo = torch.from_numpy(poff.view(np.int64)).to(dev)
    qn = torch.from_numpy(pnodes.view(np.int32)).to(dev)
    pest = torch.empty(poff.size - 1, dtype=torch.float64, device=dev)
    sk.skim_query_batch(ranks, size, n, k, ell, qo, qn, pest, mode=1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sk.skim_query_batch(ranks, size, n, k, ell, qo, qn, pest, mode=1)
    torch.cuda.synchronize()
    plain = (poff.size - 1) / (time.perf_counter() - t)
    plain_same = bool(np.array_equal(pest.cpu().numpy(), reference(poff, pnodes)))
    out["plain_queries_per_s"] = plain
    out["plain_identical_to_batch"] = plain_same

    # capacity: offered loads above the plain rate, then saturation
    sweep = []
    soff, snodes = uniform_query_sets(sweep_queries, n, cfg["qseed"] + 3, 1, 512)
    want = reference(soff, snodes)
    for rate in (500_000.0, 2_000_000.0, None):
        if rate is None:
            a = np.zeros(sweep_queries)
        else:
            a = np.cumsum(np.random.default_rng(cfg["qseed"] + 4).exponential(1.0 / rate,
                                                                              sweep_queries))
        srv = sk.Server(ranks, size, n, k, ell, budget_bytes=256 << 20, max_batch=8192,
                        streams=4)
        try:
            t = time.perf_counter()
            e, st, lt, rt = srv.replay(soff, snodes, a)
            wall = time.perf_counter() - t
        finally:
            srv.close()
        ok = bool(np.array_equal(e, want) and (st == 0).all())
        sweep.append({"offered_per_s": rate if rate is not None else "all at t=0",
                      "completed_queries_per_s": sweep_queries / wall,
                      "p50_us": float(np.percentile(lt, 50)),
                      "p99_us": float(np.percentile(lt, 99)), "admission_retries": rt,
                      "identical_to_batch": ok})
        log(f"serving sweep {sweep[-1]}")
        if not ok:
            break
    out["capacity_sweep"] = {"queries_per_point": sweep_queries, "points": sweep}
    best = max(p["completed_queries_per_s"] for p in sweep)
    out["served_capacity_queries_per_s"] = best
    out["served_over_plain"] = best / plain
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chung-lu-1m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="build only (no query/SKIM legs)")
    ap.add_argument("--no-rmat", action="store_true", help="skip the rmat-24 build leg")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the build with the default launch shapes (no autotuning)")
    ap.add_argument("--tune-cache", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                         "_build", "tune_cache.txt"),
                    help="file of cached autotuner choices (keyed by device and configuration)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB copy (for PMC byte calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1408_6282_amd as sk
    from workloads.configs import make_config, make_graph
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    sk.load_library()
    cfg = make_config(args.workload)
    log(f"generating {args.workload}")
    g = make_graph(cfg)
    cnt = oracle_counters(args.workload, g, cfg)
    log(f"oracle counters {cnt}")

    sec, work, kms, klaunch, sec_events, tuning, parity, per_kernel = bench_build(args, torch, sk,
                                                                                  g, cfg)
    value = cnt["w_live"] / sec
    alg_bytes = algorithmic_bytes_search(cnt)
    floor = algorithmic_bytes_build(cnt, g.n, cfg["k"])
    roof = None
    if klaunch:
        per_launch_bytes = alg_bytes * args.steps / klaunch
        avg_s = kms / klaunch / 1e3
        achieved = per_launch_bytes / avg_s / 1e9
        per_build = measured_traffic(args.workload)
        # per launch like `achieved`: this run's launches share the build's bytes
        traffic = None if per_build is None else per_build * args.steps / klaunch
        ra = random_access_rates(torch)
        # the searches' random accesses at the rates plain gathers and atomics
        # reach: one pair-record read per scan, one CAS per accepted visit
        floor_s = work["scans"] / ra["gather_per_s"] + work["visits"] / ra["atomic_add_per_s"]
        ra.update({"scans_per_step": work["scans"], "visits_per_step": work["visits"],
                   "search_floor_ms": floor_s * 1e3,
                   "search_floor_over_measured": floor_s / (kms / args.steps / 1e3)})
        log(f"random access {ra}")
        roof = {"bound": "hbm", "kernel": DOMINANT, "kernels": per_kernel,
                "random_access": ra,
                "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "launches_per_step": klaunch / args.steps, "avg_launch_us": avg_s * 1e6,
                "kernel_ms_per_step": kms / args.steps,
                "ms_per_step_with_kernel_events": sec_events * 1e3,
                "algorithmic_bytes_per_step": alg_bytes,
                "traffic_over_algorithmic": None if traffic is None else traffic / per_launch_bytes,
                "visit_model_bytes_per_step": visit_model_bytes(cnt),
                "build_floor_bytes": floor,
                "build_floor_ms": floor / (HBM_PEAK_GBS * 1e9) * 1e3,
                "build_floor_over_measured": floor / (HBM_PEAK_GBS * 1e9) / sec}
    out = {
        "metric": METRIC, "value": value, "unit": "live-edge traversals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": "Chung-Lu power law, gamma 2.1",
                   "n": g.n, "m": g.m, "ell": cfg["ell"], "k": cfg["k"], "seed": cfg["seed"],
                   "probabilities": "weighted cascade 1/indeg(head)",
                   "parallelism": "single GPU"},
        "parity": parity,
        "parity_check": "SHA-256 of the last timed build's sketches, sizes and estimates against "
                        "the oracle's stored digests (tests/golden)",
        "oracle_counters": cnt, "device_work": work, "roofline": roof,
        "build_params": sk.skim_get_build_params(), "autotune": tuning,
    }
    if not args.no_extras:
        log("queries")
        out["queries"] = bench_queries(torch, sk)
        log("skim")
        out["skim"] = bench_skim(torch, sk)
        if args.workload == "chung-lu-1m":
            log("skim on chung-lu-1m")
            out["skim"]["chung_lu_1m_wc"] = bench_skim_1m(torch, sk, g, cfg)
        log("oracle quality")
        out["oracle_quality"] = bench_oracle_quality(torch, sk, g, cfg)
        log("ic-model sketches")
        out["ic_sketches"] = bench_ic(torch, sk)
        log("error against the ic model")
        out["error_vs_ell"] = bench_error_vs_ell(torch, sk)
        log("serving")
        out["serving"] = bench_serving(torch, sk)
        if not args.no_rmat:
            out["rmat_24"] = bench_rmat(torch, sk)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(g, cfg)
        if not args.no_extras:
            log("oracle times of the query and SKIM workloads")
            out["oracle_times"] = oracle_times()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
