"""Write the oracle's algorithmic work counters and result digests of the
bench workloads.

Runs the CPU oracle's Algorithm 2 (Section 5.2) on the seeded synthetic graph
of each workload and stores:

* its exact counters: rank insertions N_ins, live-edge traversals W_live,
  N_exp and C_min, with a checksum of the graph.  The bench reads these as
  the algorithmic numerators of its throughput and roofline figures (never
  the kernel's own counts);
* SHA-256 digests of its results: the sketches (n x k uint64, ascending,
  UINT64_MAX padding, little-endian), the sizes (n uint32) and the estimates
  (n float64, the oracle's estimator on those sketches).  The full-size GPU
  parity tests and the bench compare the GPU's outputs with these digests,
  so the oracle need not be rerun at full size on the GPU host.

Only the oracle runs here: no value comes from the HIP library.

    python tests/golden/make_counters.py [--threads T] [workload[@ell] ...]
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads.configs import graph_sha256, make_config, make_graph  # noqa: E402


def array_digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8)).hexdigest()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main(names, threads):
    for spec in names:
        # "workload" or "workload@ell": the same graph with another l
        name, _, ell = spec.partition("@")
        cfg = make_config(name)
        if ell:
            cfg = dict(cfg, ell=int(ell))
        g = make_graph(cfg)
        t = time.time()
        R, S, cnt = oracle.build_alg2(g, cfg["seed"], cfg["ell"], cfg["k"], threads=threads)
        secs = time.time() - t
        E = oracle.estimates(R, S, cfg["k"], cfg["ell"])
        out = {"workload": name, "n": g.n, "m": g.m, "ell": cfg["ell"], "k": cfg["k"],
               "seed": cfg["seed"], "graph_sha256": graph_sha256(g), "counters": cnt,
               "digests": {"ranks_sha256": array_digest(R.astype(np.uint64)),
                           "size_sha256": array_digest(S.astype(np.uint32)),
                           "est_sha256": array_digest(E.astype(np.float64))},
               "oracle_seconds": round(secs, 2), "oracle_threads": threads,
               "oracle_cpu": cpu_model(), "source": "oracle.build_alg2"}
        tag = name.replace('-', '_') + (f"_l{ell}" if ell else "")
        path = os.path.join(HERE, f"{tag}_counters.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(path, cnt, out["digests"], f"{secs:.1f} s", flush=True)
        del R, S, E, g


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("names", nargs="*")
    a = ap.parse_args()
    main(a.names or ["chung-lu-1m", "tiny-ic"], a.threads)
