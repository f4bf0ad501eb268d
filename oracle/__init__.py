"""Python access to the CPU oracle (``skim_oracle.c``).

TEST INFRASTRUCTURE ONLY: the reference the HIP library is checked against.
Only the tests, the smoke check and the bench's CPU-baseline leg may import
this package.  It shares no code with the HIP path.

Every function takes a ``workloads.Graph``-like object (n, row_ptr, col, thr)
and numpy arrays; results come back as numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "skim_oracle.c")
_LIB = os.path.join(_HERE, "libskim_oracle.so")

UINT64_MAX = np.uint64(0xFFFFFFFFFFFFFFFF)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE doubles: no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-pthread",
                               "-fno-fast-math", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class BuildCounters(C.Structure):
    _fields_ = [("n_ins", C.c_uint64), ("w_live", C.c_uint64),
                ("n_exp", C.c_uint64), ("c_min", C.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class SkimCounters(C.Structure):
    _fields_ = [("insertions", C.c_uint64), ("pairs_scanned", C.c_uint64),
                ("reverse_bfs", C.c_uint64), ("covered", C.c_uint64),
                ("decrements", C.c_uint64), ("fallback", C.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lib = None
P64 = C.POINTER(C.c_uint64)
P32 = C.POINTER(C.c_uint32)
PI32 = C.POINTER(C.c_int32)
PD = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        lib.or_sm64.restype = C.c_uint64
        lib.or_sm64.argtypes = [C.c_uint64, C.c_uint64]
        lib.or_rank.restype = C.c_uint64
        lib.or_rank.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32]
        lib.or_live.restype = C.c_int
        lib.or_live.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                C.c_uint32]
        lib.or_ranks.restype = None
        lib.or_ranks.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, P64]
        lib.or_pair_ranks.restype = None
        lib.or_pair_ranks.argtypes = [C.c_uint64, C.c_uint64, P64, P64]
        lib.or_live_batch.restype = None
        lib.or_live_batch.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, P32, P32, P32, P32,
                                      C.POINTER(C.c_uint8)]
        lib.or_influence.restype = C.c_uint64
        lib.or_influence.argtypes = [C.c_uint32, P64, P32, P32, C.c_uint64, C.c_uint32, P32,
                                     C.c_uint64, P64]
        lib.or_sketch_brute.restype = None
        lib.or_sketch_brute.argtypes = [C.c_uint32, P64, P32, P32, C.c_uint64, C.c_uint32,
                                        C.c_uint32, P32, C.c_uint64, P64, P32, P64]
        lib.or_sketch_brute_budget.restype = None
        lib.or_sketch_brute_budget.argtypes = [C.c_uint32, P64, P32, P32, C.c_uint64, C.c_uint32,
                                               C.c_uint32, P32, C.c_uint64, C.c_uint64,
                                               C.c_uint32, P64, P32, P64, C.POINTER(C.c_uint8)]
        lib.or_build_alg2.restype = C.c_int
        lib.or_build_alg2.argtypes = [C.c_uint32, P64, P32, P32, C.c_uint64, C.c_uint32,
                                      C.c_uint32, C.c_uint32, P64, P32, C.POINTER(BuildCounters)]
        lib.or_estimates.restype = None
        lib.or_estimates.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, P64, P32, PD]
        for fn in (lib.or_union_query, lib.or_ck_query):
            fn.restype = None
            fn.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, P64, P32, C.c_uint64, P64, P32,
                           PD, PI32]
        lib.or_skim.restype = C.c_int
        lib.or_skim.argtypes = [C.c_uint32, P64, P32, P32, C.c_uint64, C.c_uint32, C.c_uint32,
                                C.c_uint32, P32, P64, P64, P32, C.POINTER(SkimCounters)]
        lib.or_ic_live.restype = C.c_int
        lib.or_ic_live.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                   C.c_uint32]
        lib.or_ic_order.restype = None
        lib.or_ic_order.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, P32]
        lib.or_ic_sketches.restype = C.c_int
        lib.or_ic_sketches.argtypes = [C.c_uint32, P64, P32, P32, C.c_uint32, C.c_uint64, P32,
                                       PD, P64]
        lib.or_ic_union_query.restype = None
        lib.or_ic_union_query.argtypes = [C.c_uint32, C.c_uint32, P32, C.c_uint64, P64, P32,
                                          C.c_uint32, PD, PI32]
        lib.or_perm_positions.restype = None
        lib.or_perm_positions.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, P64]
        lib.or_build_alg2_table.restype = C.c_int
        lib.or_build_alg2_table.argtypes = [C.c_uint32, P64, P32, P32, C.c_uint64, C.c_uint32,
                                            C.c_uint32, P64, C.c_uint32, P64, P32,
                                            C.POINTER(BuildCounters)]
        lib.or_sketch_brute_table.restype = None
        lib.or_sketch_brute_table.argtypes = [C.c_uint32, P64, P32, P32, C.c_uint64, C.c_uint32,
                                              C.c_uint32, P64, P32, C.c_uint64, P64, P32]
        lib.or_perm_estimates.restype = None
        lib.or_perm_estimates.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, P64, P32, PD]
        lib.or_perm_union_query.restype = None
        lib.or_perm_union_query.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, P64, P32,
                                            C.c_uint64, P64, P32, C.c_uint32, PD, PI32]
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _g(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    thr = np.ascontiguousarray(g.thr, dtype=np.uint32)
    if col.size == 0:  # keep valid pointers for empty graphs
        col = np.zeros(1, dtype=np.uint32)
        thr = np.zeros(1, dtype=np.uint32)
    return rp, col, thr


def sm64(seed: int, counter: int) -> int:
    return int(_load().or_sm64(seed, counter))


def rank(seed: int, v: int, i: int) -> int:
    return int(_load().or_rank(seed, v, i))


def live(seed: int, n: int, u: int, v: int, i: int, thr: int) -> bool:
    return bool(_load().or_live(seed, n, u, v, i, thr))


def ranks(seed: int, n: int, ell: int) -> np.ndarray:
    """All ranks r(v, i) as an [n, l] uint64 array."""
    out = np.empty(n * ell, dtype=np.uint64)
    _load().or_ranks(seed, n, ell, _p(out, P64))
    return out.reshape(n, ell)


def live_batch(seed: int, n: int, u, v, inst, thr) -> np.ndarray:
    """Live-edge coins for arrays of (u, v, i, thr)."""
    u = np.ascontiguousarray(u, dtype=np.uint32)
    v = np.ascontiguousarray(v, dtype=np.uint32)
    inst = np.ascontiguousarray(inst, dtype=np.uint32)
    thr = np.ascontiguousarray(np.broadcast_to(thr, u.shape), dtype=np.uint32)
    out = np.empty(u.size, dtype=np.uint8)
    _load().or_live_batch(seed, n, u.size, _p(u, P32), _p(v, P32), _p(inst, P32), _p(thr, P32),
                          out.ctypes.data_as(C.POINTER(C.c_uint8)))
    return out.astype(bool)


def influence(g, seed: int, ell: int, S, per_instance: bool = False):
    """l * Inf({G^(i)}, S) as an exact integer (and per-instance counts)."""
    rp, col, thr = _g(g)
    S = np.ascontiguousarray(S, dtype=np.uint32)
    Sp = S if S.size else np.zeros(1, dtype=np.uint32)
    per = np.zeros(max(ell, 1), dtype=np.uint64)
    tot = _load().or_influence(g.n, _p(rp, P64), _p(col, P32), _p(thr, P32), seed, ell,
                               _p(Sp, P32), S.size, _p(per, P64))
    return (int(tot), per[:ell]) if per_instance else int(tot)


def pair_ranks(seed: int, pairs) -> np.ndarray:
    """r(v, i) for pair ids p = 64 v + i (Section 3's ranks)."""
    p = np.ascontiguousarray(pairs, dtype=np.uint64)
    out = np.empty(p.size, dtype=np.uint64)
    if p.size:
        _load().or_pair_ranks(seed & ((1 << 64) - 1), p.size, _p(p, P64), _p(out, P64))
    return out


def sketch_brute(g, seed: int, ell: int, k: int, nodes=None, budget: int | None = None,
                 threads: int | None = None):
    """Sketches by the plain definition, for the given nodes (default all).

    With `budget`, a node whose forward searches (over all l instances) would
    scan more out-edges than that is left out; returns (ranks, size, reach,
    ok) then, ok[j] = False for a node left out (its rows are undefined).
    """
    rp, col, thr = _g(g)
    nodes = np.arange(g.n, dtype=np.uint32) if nodes is None else \
        np.ascontiguousarray(nodes, dtype=np.uint32)
    ranks = np.empty(nodes.size * k, dtype=np.uint64)
    size = np.empty(nodes.size, dtype=np.uint32)
    reach = np.empty(nodes.size, dtype=np.uint64)
    ok = np.ones(nodes.size, dtype=np.uint8)
    nthreads = threads or min(16, os.cpu_count() or 1)
    _load().or_sketch_brute_budget(g.n, _p(rp, P64), _p(col, P32), _p(thr, P32), seed, ell, k,
                                   _p(nodes, P32), nodes.size,
                                   (1 << 64) - 1 if budget is None else int(budget),
                                   nthreads if budget is not None or threads else 1,
                                   _p(ranks, P64), _p(size, P32), _p(reach, P64),
                                   ok.ctypes.data_as(C.POINTER(C.c_uint8)))
    if budget is None:
        return ranks.reshape(nodes.size, k), size, reach
    return ranks.reshape(nodes.size, k), size, reach, ok.astype(bool)


def build_alg2(g, seed: int, ell: int, k: int, threads: int | None = None):
    """Sketches of every node by Algorithm 2 -> (ranks[n,k], size[n], counters)."""
    rp, col, thr = _g(g)
    ranks = np.empty(g.n * k, dtype=np.uint64)
    size = np.empty(g.n, dtype=np.uint32)
    cnt = BuildCounters()
    if threads is None:
        threads = os.cpu_count() or 1
    rc = _load().or_build_alg2(g.n, _p(rp, P64), _p(col, P32), _p(thr, P32), seed, ell, k,
                               threads, _p(ranks, P64), _p(size, P32), C.byref(cnt))
    if rc != 0:
        raise ValueError("or_build_alg2: bad arguments")
    return ranks.reshape(g.n, k), size, cnt.as_dict()


def estimates(ranks: np.ndarray, size: np.ndarray, k: int, ell: int) -> np.ndarray:
    n = size.shape[0]
    r = np.ascontiguousarray(ranks, dtype=np.uint64).reshape(-1)
    s = np.ascontiguousarray(size, dtype=np.uint32)
    out = np.empty(n, dtype=np.float64)
    _load().or_estimates(n, k, ell, _p(r, P64), _p(s, P32), _p(out, PD))
    return out


def _query(fn, ranks, size, k, ell, offsets, nodes):
    n = size.shape[0]
    r = np.ascontiguousarray(ranks, dtype=np.uint64).reshape(-1)
    s = np.ascontiguousarray(size, dtype=np.uint32)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    nd = np.ascontiguousarray(nodes, dtype=np.uint32)
    if nd.size == 0:
        nd = np.zeros(1, dtype=np.uint32)
    Q = off.size - 1
    est = np.empty(max(Q, 1), dtype=np.float64)
    st = np.empty(max(Q, 1), dtype=np.int32)
    fn(n, k, ell, _p(r, P64), _p(s, P32), Q, _p(off, P64), _p(nd, P32), _p(est, PD),
       _p(st, PI32))
    return est[:Q], st[:Q]


def union_query(ranks, size, k, ell, offsets, nodes):
    """Bottom-k-of-the-union estimates (divided by l) and per-query status."""
    return _query(_load().or_union_query, ranks, size, k, ell, offsets, nodes)


def ck_query(ranks, size, k, ell, offsets, nodes):
    """Cohen-Kaplan union estimates (divided by l) and per-query status."""
    return _query(_load().or_ck_query, ranks, size, k, ell, offsets, nodes)


def skim(g, seed: int, ell: int, k: int, s: int, records: bool = False):
    """SKIM seeds, exact newly-covered pair counts, counters.

    With ``records`` also the per-seed tau (uint64 rank of the pair that filled
    the seed's sketch; 2^64-1 for an exhaustion seed) and second largest sketch
    k' of the adaptive error estimate: (seeds, gains, tau, second, counters).
    """
    rp, col, thr = _g(g)
    seeds = np.zeros(max(s, 1), dtype=np.uint32)
    gain = np.zeros(max(s, 1), dtype=np.uint64)
    tau = np.zeros(max(s, 1), dtype=np.uint64)
    second = np.zeros(max(s, 1), dtype=np.uint32)
    cnt = SkimCounters()
    rc = _load().or_skim(g.n, _p(rp, P64), _p(col, P32), _p(thr, P32), seed, ell, k, s,
                         _p(seeds, P32), _p(gain, P64), _p(tau, P64), _p(second, P32),
                         C.byref(cnt))
    if rc == -1:
        raise ValueError("or_skim: bad arguments")
    if rc == -2:
        raise AssertionError("or_skim: reverse search met a covered pair")
    if records:
        return seeds[:s], gain[:s], tau[:s], second[:s], cnt.as_dict()
    return seeds[:s], gain[:s], cnt.as_dict()


def ic_live(seed: int, n: int, u: int, w: int, t: int, thr: int) -> bool:
    """Is edge (u -> w) live in the IC-model instance of position t (>= 1)?"""
    return bool(_load().or_ic_live(seed & 0xFFFFFFFFFFFFFFFF, n, u, w, t, thr))


def ic_order(seed: int, n: int, k: int) -> np.ndarray:
    """node_at[t - 1]: the node at structured permutation position t, t = 1..k n."""
    out = np.zeros(max(k * n, 1), dtype=np.uint32)
    _load().or_ic_order(seed & 0xFFFFFFFFFFFFFFFF, n, k, _p(out, P32))
    return out[:k * n]


def ic_sketches(g, k: int, seed: int):
    """IC-model sketches: positions [n, k] (uint32, ascending), estimates
    n (k - 1) / (T - 1) [n], and the number of (position, node) visits."""
    rp, col, thr = _g(g)
    pos = np.zeros(max(g.n * k, 1), dtype=np.uint32)
    est = np.zeros(max(g.n, 1))
    visits = np.zeros(1, dtype=np.uint64)
    rc = _load().or_ic_sketches(g.n, _p(rp, P64), _p(col, P32), _p(thr, P32), k,
                                seed & 0xFFFFFFFFFFFFFFFF, _p(pos, P32), _p(est, PD),
                                _p(visits, P64))
    if rc == -1:
        raise ValueError("or_ic_sketches: bad arguments")
    if rc == -2:
        raise AssertionError("or_ic_sketches: a node holds fewer than k positions")
    return pos[:g.n * k].reshape(g.n, k), est[:g.n], int(visits[0])


def ic_union_query(pos, n: int, k: int, offsets, nodes, estimator: int = 0):
    """Union estimates over IC-model sketches (estimator 0 bottom-k, 1
    Cohen-Kaplan) and per-query status."""
    pos = np.ascontiguousarray(pos, dtype=np.uint32).reshape(-1)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    nd = np.ascontiguousarray(nodes, dtype=np.uint32)
    q = off.size - 1
    est = np.zeros(max(q, 1))
    st = np.zeros(max(q, 1), dtype=np.int32)
    ndp = nd if nd.size else np.zeros(1, dtype=np.uint32)
    _load().or_ic_union_query(n, k, _p(pos, P32), q, _p(off, P64), _p(ndp, P32), estimator,
                              _p(est, PD), _p(st, PI32))
    return est[:q], st[:q]


# ---------------------------------------------- structured permutation ranks

def perm_positions(seed: int, n: int, ell: int) -> np.ndarray:
    """[n, 64] uint64: the position (1..n l) of pair (v, i) in the structured
    permutation of Section 3.1 (0 for i >= l)."""
    out = np.zeros(n * 64, dtype=np.uint64)
    _load().or_perm_positions(seed, n, ell, _p(out, P64))
    return out.reshape(n, 64)


def build_alg2_perm(g, seed: int, ell: int, k: int, threads: int | None = None):
    """Algorithm 2 with permutation positions as ranks -> (sketches[n, k] of
    positions, size[n], counters)."""
    rp, col, thr = _g(g)
    pos = np.ascontiguousarray(perm_positions(seed, g.n, ell).reshape(-1))
    ranks = np.empty(g.n * k, dtype=np.uint64)
    size = np.empty(g.n, dtype=np.uint32)
    cnt = BuildCounters()
    if threads is None:
        threads = os.cpu_count() or 1
    rc = _load().or_build_alg2_table(g.n, _p(rp, P64), _p(col, P32), _p(thr, P32), seed, ell, k,
                                     _p(pos, P64), threads, _p(ranks, P64), _p(size, P32),
                                     C.byref(cnt))
    if rc != 0:
        raise ValueError("or_build_alg2_table: bad arguments")
    return ranks.reshape(g.n, k), size, cnt.as_dict()


def sketch_brute_perm(g, seed: int, ell: int, k: int, nodes=None):
    """The definition (forward search per node and instance) with permutation
    positions as ranks -> (sketches[len(nodes), k], size)."""
    rp, col, thr = _g(g)
    pos = np.ascontiguousarray(perm_positions(seed, g.n, ell).reshape(-1))
    nodes = np.arange(g.n, dtype=np.uint32) if nodes is None else \
        np.ascontiguousarray(nodes, dtype=np.uint32)
    ranks = np.empty(max(nodes.size, 1) * k, dtype=np.uint64)
    size = np.empty(max(nodes.size, 1), dtype=np.uint32)
    _load().or_sketch_brute_table(g.n, _p(rp, P64), _p(col, P32), _p(thr, P32), seed, ell, k,
                                  _p(pos, P64), _p(nodes, P32), nodes.size, _p(ranks, P64),
                                  _p(size, P32))
    return ranks[:nodes.size * k].reshape(nodes.size, k), size[:nodes.size]


def perm_estimates(ranks, size, n: int, k: int, ell: int) -> np.ndarray:
    r = np.ascontiguousarray(ranks, dtype=np.uint64).reshape(-1)
    sz = np.ascontiguousarray(size, dtype=np.uint32)
    out = np.empty(n)
    _load().or_perm_estimates(n, k, ell, _p(r, P64), _p(sz, P32), _p(out, PD))
    return out


def perm_union_query(ranks, size, n: int, k: int, ell: int, offsets, nodes, estimator: int = 0):
    r = np.ascontiguousarray(ranks, dtype=np.uint64).reshape(-1)
    sz = np.ascontiguousarray(size, dtype=np.uint32)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    nd = np.ascontiguousarray(nodes, dtype=np.uint32)
    q = off.size - 1
    est = np.zeros(max(q, 1))
    st = np.zeros(max(q, 1), dtype=np.int32)
    ndp = nd if nd.size else np.zeros(1, dtype=np.uint32)
    _load().or_perm_union_query(n, k, ell, _p(r, P64), _p(sz, P32), q, _p(off, P64),
                                _p(ndp, P32), estimator, _p(est, PD), _p(st, PI32))
    return est[:q], st[:q]
