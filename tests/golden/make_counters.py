"""Write the oracle's algorithmic work counters of the bench workloads.

Runs the CPU oracle's Algorithm 2 (Section 5.2) on the seeded synthetic graph
of each workload and stores its exact counters: rank insertions N_ins,
live-edge traversals W_live, N_exp and C_min, with a checksum of the graph.
The bench reads these as the algorithmic numerators of its throughput and
roofline figures (never the kernel's own counts).

    python tests/golden/make_counters.py [workload ...]
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads.configs import make_config, make_graph  # noqa: E402


def graph_digest(g) -> str:
    h = hashlib.sha256()
    for a in (g.row_ptr, g.col, g.thr):
        h.update(memoryview(a).cast("B"))
    return h.hexdigest()


def main(names):
    for name in names:
        cfg = make_config(name)
        g = make_graph(cfg)
        t = time.time()
        _, _, cnt = oracle.build_alg2(g, cfg["seed"], cfg["ell"], cfg["k"])
        out = {"workload": name, "n": g.n, "m": g.m, "ell": cfg["ell"], "k": cfg["k"],
               "seed": cfg["seed"], "graph_sha256": graph_digest(g), "counters": cnt,
               "oracle_seconds": round(time.time() - t, 2), "source": "oracle.build_alg2"}
        path = os.path.join(HERE, f"{name.replace('-', '_')}_counters.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(path, cnt)


if __name__ == "__main__":
    main(sys.argv[1:] or ["chung-lu-1m", "tiny-ic"])
