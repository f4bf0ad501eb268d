"""Synthetic directed graphs shaped like the paper's workloads (Section 6).

The paper measures on SNAP / WebGraph social, collaboration and web networks,
which are heavy-tailed.  Those datasets are not available here, so seeded
synthetic graphs stand in for them:

* Erdos-Renyi: exactly m distinct ordered pairs (u, v), u != v.
* Chung-Lu: expected degrees w_i ~ (i+1)^(-1/(gamma-1)) for in- and
  out-degrees, each behind its own seeded node permutation; edges are sampled
  source ~ out-weight, head ~ in-weight, self-loops and duplicates dropped,
  and a seeded subset of exactly m distinct edges kept.
* R-MAT: 2^scale nodes, a fixed number of recursive quadrant samples with
  probabilities (a, b, c, d) (float32 uniforms), a seeded node permutation,
  then self-loops and duplicates dropped (the final edge count is reported,
  not topped up).

Every graph is returned as a forward CSR (out-edges): row_ptr uint64[n+1],
col uint32[m] with strictly increasing heads inside each row, no self-loops,
no duplicates.  Per-edge probabilities are uint32 thresholds aligned with col.

Edge-probability schemes (Section 6, the IC setup): uniform p, weighted cascade
p_uv = 1 / indeg(v), and the trivalency scheme {0.1, 0.01, 0.001}.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

UINT32_MAX = np.uint64(0xFFFFFFFF)


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # uint64[n+1]
    col: np.ndarray      # uint32[m]
    thr: np.ndarray      # uint32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def edges(self):
        """(src, dst) arrays in CSR order."""
        deg = np.diff(self.row_ptr.astype(np.int64))
        src = np.repeat(np.arange(self.n, dtype=np.uint32), deg)
        return src, self.col

    def in_degree(self) -> np.ndarray:
        return np.bincount(self.col, minlength=self.n).astype(np.int64)


def _csr_from_keys(n: int, keys: np.ndarray):
    """Sorted unique keys src*n+dst -> (row_ptr, col)."""
    keys = np.asarray(keys, dtype=np.uint64)
    src = (keys // np.uint64(n)).astype(np.int64)
    dst = (keys % np.uint64(n)).astype(np.uint32)
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, dst


def from_edges(n: int, src, dst, thr=None, name: str = "") -> Graph:
    """Build a Graph from explicit edge lists (used by small tests).

    Duplicates and self-loops are rejected, not silently dropped, so that a
    test always knows the exact graph it built.  ``thr`` may be a scalar or an
    array aligned with (src, dst); it is permuted into CSR order.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if src.shape != dst.shape:
        raise ValueError("src/dst length mismatch")
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("node id out of range")
    if np.any(src == dst):
        raise ValueError("self-loop")
    keys = src.astype(np.uint64) * np.uint64(n) + dst.astype(np.uint64)
    order = np.argsort(keys, kind="stable")
    skeys = keys[order]
    if skeys.size > 1 and np.any(skeys[1:] == skeys[:-1]):
        raise ValueError("duplicate edge")
    row_ptr, col = _csr_from_keys(n, skeys)
    if thr is None:
        t = np.full(col.shape[0], 0xFFFFFFFF, dtype=np.uint32)
    elif np.isscalar(thr):
        t = np.full(col.shape[0], int(thr), dtype=np.uint32)
    else:
        t = np.asarray(thr, dtype=np.uint32)[order]
    return Graph(n, row_ptr, col.astype(np.uint32), t, name)


def uniform_thresholds(m: int, denom: int) -> np.ndarray:
    """Uniform scheme p = 1/denom for every edge: thr = (2^32-1) // denom."""
    if denom < 1:
        raise ValueError("denom >= 1")
    return np.full(m, 0xFFFFFFFF // int(denom), dtype=np.uint32)


def wc_thresholds(row_ptr: np.ndarray, col: np.ndarray, n: int) -> np.ndarray:
    """Weighted cascade: p_uv = 1 / indeg(v), thr = (2^32-1) // indeg(v)."""
    indeg = np.bincount(col, minlength=n).astype(np.uint64)
    d = indeg[col]
    return (UINT32_MAX // d).astype(np.uint32)


def trivalency_thresholds(m: int, seed: int) -> np.ndarray:
    """Trivalency: p drawn uniformly from {0.1, 0.01, 0.001} per edge."""
    rng = np.random.Generator(np.random.PCG64(seed))
    choices = np.array([0xFFFFFFFF // 10, 0xFFFFFFFF // 100, 0xFFFFFFFF // 1000],
                       dtype=np.uint32)
    return choices[rng.integers(0, 3, size=m)]


def er_graph(n: int, m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Exactly m distinct ordered pairs (u, v) with u != v, uniformly."""
    if m > n * (n - 1):
        raise ValueError("m too large")
    rng = np.random.Generator(np.random.PCG64(seed))
    code = rng.choice(n * (n - 1), size=m, replace=False).astype(np.int64)
    u = code // (n - 1)
    v = code % (n - 1)
    v = v + (v >= u)  # skip the diagonal
    keys = np.sort(u.astype(np.uint64) * np.uint64(n) + v.astype(np.uint64))
    return _csr_from_keys(n, keys)


def _sample_powerlaw_rank(rng, n: int, expo: float, size: int) -> np.ndarray:
    """Rank j in [0, n) with P(j) ~ (j+1)^-expo, by inverting the continuous
    cumulative weight int_0^x (t+1)^-expo dt (a discretised power law)."""
    u = rng.random(size)
    one = 1.0 - expo
    top = (n + 1.0) ** one - 1.0
    x = np.power(1.0 + u * top, 1.0 / one) - 1.0
    return np.minimum(x.astype(np.int64), n - 1)


def chung_lu_graph(n: int, m: int, gamma: float, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Chung-Lu directed graph with power-law in/out expected degrees.

    Out- and in-weights follow (j+1)^(-1/(gamma-1)) over ranks j, mapped to
    nodes by two independent seeded permutations.  Edges are sampled
    source ~ out-weight, head ~ in-weight; self-loops and duplicates are
    dropped; a seeded random subset of exactly m distinct edges is kept.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    expo = 1.0 / (gamma - 1.0)
    perm_out = rng.permutation(n).astype(np.uint64)
    perm_in = rng.permutation(n).astype(np.uint64)
    keys = np.empty(0, dtype=np.uint64)
    batch = int(m * 1.35) + 1024
    while True:
        src = perm_out[_sample_powerlaw_rank(rng, n, expo, batch)]
        dst = perm_in[_sample_powerlaw_rank(rng, n, expo, batch)]
        new = (src * np.uint64(n) + dst)[src != dst]
        keys = np.unique(np.concatenate([keys, new]))
        if keys.size >= m:
            break
        batch = int((m - keys.size) * 2) + 1024
    if keys.size > m:
        keep = rng.choice(keys.size, size=m, replace=False)
        keys = np.sort(keys[keep])
    return _csr_from_keys(n, keys)


def _rmat_chunk(ss, cnt: int, scale: int, abcd, perm: np.ndarray, nb: int) -> list:
    """One chunk of R-MAT samples from its own seed sequence: permuted, no
    self-loops, deduplicated, split into `nb` buckets by the top bits of the
    source (each bucket sorted)."""
    a, b, c, _ = abcd
    rng = np.random.Generator(np.random.PCG64(ss))
    src = np.zeros(cnt, dtype=np.uint32)
    dst = np.zeros(cnt, dtype=np.uint32)
    f_ab, f_abc, f_a = np.float32(a + b), np.float32(a + b + c), np.float32(a)
    for _ in range(scale):
        u = rng.random(cnt, dtype=np.float32)
        down = u >= f_ab                                   # quadrant c or d
        right = np.where(down, u >= f_abc, u >= f_a)       # quadrant b or d
        src = (src << np.uint32(1)) | down.astype(np.uint32)
        dst = (dst << np.uint32(1)) | right.astype(np.uint32)
    src = perm[src]
    dst = perm[dst]
    ok = src != dst
    src = src[ok]
    keys = (src.astype(np.uint64) << np.uint64(scale)) | dst[ok].astype(np.uint64)
    shift = max(scale - (nb.bit_length() - 1), 0)
    bucket = (src >> np.uint32(shift)).astype(np.int64)
    order = np.argsort(bucket, kind="stable")
    keys, bucket = keys[order], bucket[order]
    bounds = np.searchsorted(bucket, np.arange(nb + 1))
    return [np.unique(keys[bounds[j]:bounds[j + 1]]) for j in range(nb)]


def rmat_graph(scale: int, samples: int, abcd, seed: int,
               chunks: int = 64, threads: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """R-MAT: `samples` recursive quadrant draws with probabilities (a, b, c,
    d), a seeded node permutation, self-loops and duplicates dropped.

    The samples come in `chunks` fixed chunks, chunk j drawn from the j-th
    child of the seed sequence, so the graph does not depend on how many
    threads generate it.  Threads work on chunks, then on source buckets
    (numpy releases the interpreter lock in its bulk kernels).
    """
    import os
    from concurrent.futures import ThreadPoolExecutor
    n = 1 << scale
    root = np.random.SeedSequence(seed)
    perm_ss, *chunk_ss = root.spawn(chunks + 1)
    perm = np.random.Generator(np.random.PCG64(perm_ss)).permutation(n).astype(np.uint32)
    sizes = [samples // chunks + (1 if j < samples % chunks else 0) for j in range(chunks)]
    nb = 16
    threads = threads or max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda j: _rmat_chunk(chunk_ss[j], sizes[j], scale, abcd, perm, nb),
                            range(chunks)))
        merged = list(ex.map(lambda b: np.unique(np.concatenate([p[b] for p in parts])),
                             range(nb)))
    del parts
    keys = np.concatenate(merged)
    return _csr_from_keys(n, keys)
