"""The five synthetic workloads, as concrete seeded inputs.

1 tiny-ic        ER n=1,000 m=8,000, uniform p=1/20, l=16, k=16, rank seed 1;
                 sketches for every node + 1,000 single-node queries.
2 chung-lu-1m    Chung-Lu n=1,000,000 m=16,000,000, gamma=2.1 in and out,
                 weighted cascade, l=64, k=64; sketches + estimates for all.
3 rmat-24        R-MAT scale 24, 2^28 samples, (.57,.19,.19,.05), trivalency,
                 l=64, k=32; sketches only.
4 batched-query  config-1 sketches, 1,000,000 lognormal(2,1) sets in [1,512].
5 served-skim    ER n=1,000 m=8,000, uniform p=1/100, l=64, k=64, 200 seeds,
                 plus a Poisson(50k/s) stream of U[1,512] sets.

``seed`` is the method's seed (ranks and live-edge coins); generator seeds are
separate and fixed here.
"""
from __future__ import annotations

from .graphs import (Graph, er_graph, chung_lu_graph, rmat_graph, uniform_thresholds,
                     wc_thresholds, trivalency_thresholds)

CONFIGS = {
    "tiny-ic": dict(kind="er", n=1000, m=8000, denom=20, ell=16, k=16, seed=1, gseed=101),
    "chung-lu-1m": dict(kind="chung_lu", n=1_000_000, m=16_000_000, gamma=2.1, ell=64, k=64,
                        seed=1, gseed=102),
    "rmat-24": dict(kind="rmat", scale=24, samples=1 << 28, abcd=(0.57, 0.19, 0.19, 0.05),
                    ell=64, k=32, seed=1, gseed=103),
    "batched-query": dict(kind="er", n=1000, m=8000, denom=20, ell=16, k=16, seed=1, gseed=101,
                          Q=1_000_000, qseed=104),
    "served-skim": dict(kind="er", n=1000, m=8000, denom=100, ell=64, k=64, seed=1, gseed=101,
                        s=200, rate=50_000.0, duration=10.0, qseed=105),
}


def make_graph(cfg: dict, scale_n: int | None = None, scale_m: int | None = None) -> Graph:
    """Materialise the graph of a config (optionally at a reduced size)."""
    kind = cfg["kind"]
    if kind == "er":
        n = scale_n or cfg["n"]
        m = scale_m or cfg["m"]
        row_ptr, col = er_graph(n, m, cfg["gseed"])
        thr = uniform_thresholds(col.shape[0], cfg["denom"])
    elif kind == "chung_lu":
        n = scale_n or cfg["n"]
        m = scale_m or cfg["m"]
        row_ptr, col = chung_lu_graph(n, m, cfg["gamma"], cfg["gseed"])
        thr = wc_thresholds(row_ptr, col, n)
    elif kind == "rmat":
        scale = cfg["scale"] if scale_n is None else int(scale_n).bit_length() - 1
        samples = cfg["samples"] if scale_m is None else scale_m
        row_ptr, col = rmat_graph(scale, samples, cfg["abcd"], cfg["gseed"])
        n = 1 << scale
        thr = trivalency_thresholds(col.shape[0], cfg["gseed"] + 1)
    else:
        raise ValueError(kind)
    return Graph(n, row_ptr, col, thr, kind)


def make_config(name: str, **overrides) -> dict:
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    cfg["name"] = name
    return cfg


def graph_sha256(g: Graph) -> str:
    """SHA-256 of a graph's arrays (row_ptr, col, thr), to tie stored results to their input."""
    import hashlib
    h = hashlib.sha256()
    for a in (g.row_ptr, g.col, g.thr):
        h.update(memoryview(a).cast("B"))
    return h.hexdigest()
