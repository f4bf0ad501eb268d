"""Write the oracle's SKIM seed sequence for a full-size workload graph.

Runs the CPU oracle's Algorithm 1 (Section 4) on the seeded synthetic graph
of a workload and stores the seeds and their exact gains (newly covered
node-instance pairs), with the oracle's counters, time and a checksum of the
graph.  The GPU parity test compares skim_greedy's sequence with it.  Only
the oracle runs here: no value comes from the HIP library.

    python tests/golden/make_skim.py WORKLOAD SEEDS
"""
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads.configs import graph_sha256, make_config, make_graph  # noqa: E402


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main(name, s):
    cfg = make_config(name)
    g = make_graph(cfg)
    t = time.time()
    seeds, gains, cnt = oracle.skim(g, cfg["seed"], cfg["ell"], cfg["k"], s)
    secs = time.time() - t
    out = {"workload": name, "n": g.n, "m": g.m, "ell": cfg["ell"], "k": cfg["k"],
           "seed": cfg["seed"], "s": s, "graph_sha256": graph_sha256(g),
           "seeds": [int(x) for x in seeds], "gain_pairs": [int(x) for x in gains],
           "counters": cnt, "oracle_seconds": round(secs, 2), "oracle_threads": 1,
           "oracle_cpu": cpu_model(), "source": "oracle.skim"}
    path = os.path.join(HERE, f"{name.replace('-', '_')}_skim.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, f"{secs:.1f} s", cnt)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]))
