"""Pins for the oracle's influence over l instances (Section 2, eqs. Inf, timedinf).

Exact cases: deterministic graphs (p = 1), no edges.  Probabilistic cases:
closed-form IC expectations and exact enumeration of every live-edge subset
(graphs with at most 10 edges); the Monte-Carlo average over instances must
lie within 5 standard errors of the exact expectation (Section 1: the average
over simulated instances is an unbiased estimate of the IC influence).
"""
from fractions import Fraction

import numpy as np
import pytest

from workloads import from_edges
from brute import exact_ic_influence, reach, random_small_graph, thr_prob

HALF = 0xFFFFFFFF // 2  # encodes p = 1/2 exactly: (2^31 - 1 + 1) / 2^32


def test_no_edges(oracle_lib):
    g = from_edges(10, [], [])
    assert oracle_lib.influence(g, 1, 16, [3]) == 16
    assert oracle_lib.influence(g, 1, 16, [3, 4, 3]) == 32  # duplicates count once
    assert oracle_lib.influence(g, 1, 16, []) == 0


def test_deterministic_graph_is_reachability(oracle_lib):
    rng = np.random.default_rng(1)
    for trial in range(20):
        n = int(rng.integers(2, 40))
        m = int(rng.integers(0, n * (n - 1) // 2 + 1))
        src, dst, _ = random_small_graph(rng, n, m, [0xFFFFFFFF])
        g = from_edges(n, src, dst, 0xFFFFFFFF)
        adj = [[] for _ in range(n)]
        for a, b in zip(src, dst):
            adj[int(a)].append(int(b))
        S = list(rng.choice(n, size=int(rng.integers(1, n + 1)), replace=False))
        ell = int(rng.integers(1, 65))
        assert oracle_lib.influence(g, trial, ell, S) == ell * len(reach(adj, S))


def _mc_mean(oracle_lib, g, S, ell=64, seeds=300):
    tot = 0
    for s in range(seeds):
        tot += oracle_lib.influence(g, 1000 + s, ell, S)
    return tot / (ell * seeds), ell * seeds


@pytest.mark.parametrize("shape", ["path", "star", "diamond", "two_cycle"])
def test_closed_forms(oracle_lib, shape):
    p = Fraction(1, 2)
    if shape == "path":      # 0 -> 1 -> 2 -> 3: 1 + p + p^2 + p^3
        g = from_edges(4, [0, 1, 2], [1, 2, 3], HALF)
        exact = 1 + p + p ** 2 + p ** 3
    elif shape == "star":    # out-star with 5 leaves: 1 + 5p
        g = from_edges(6, [0] * 5, [1, 2, 3, 4, 5], HALF)
        exact = 1 + 5 * p
    elif shape == "diamond":  # 0->1, 0->2, 1->3, 2->3: 1 + 2p + 2p^2 - p^4
        g = from_edges(4, [0, 0, 1, 2], [1, 2, 3, 3], HALF)
        exact = 1 + 2 * p + 2 * p ** 2 - p ** 4
    else:                     # 0 <-> 1: 1 + p
        g = from_edges(2, [0, 1], [1, 0], HALF)
        exact = 1 + p
    E = [(int(a), int(b), thr_prob(t)) for (a, b), t in zip(zip(*g.edges()), g.thr)]
    mean_e, var_e = exact_ic_influence(g.n, E, [0])
    assert mean_e == exact  # the enumeration itself agrees with the closed form
    mc, N = _mc_mean(oracle_lib, g, [0])
    se = float(var_e) ** 0.5 / N ** 0.5
    assert abs(mc - float(exact)) < 5 * se


def test_exact_enumeration_random(oracle_lib):
    rng = np.random.default_rng(7)
    for trial in range(6):
        n = int(rng.integers(3, 7))
        m = int(rng.integers(3, 10))
        src, dst, thr = random_small_graph(rng, n, m, [0xFFFFFFFF // 2, 0xFFFFFFFF // 3,
                                                       0xFFFFFFFF // 5, 0xFFFFFFFF])
        g = from_edges(n, src, dst, thr)
        E = [(int(a), int(b), thr_prob(t)) for (a, b), t in zip(zip(*g.edges()), g.thr)]
        S = [int(x) for x in rng.choice(n, size=int(rng.integers(1, 3)), replace=False)]
        mean_e, var_e = exact_ic_influence(n, E, S)
        mc, N = _mc_mean(oracle_lib, g, S, seeds=200)
        se = max(float(var_e), 1e-12) ** 0.5 / N ** 0.5
        assert abs(mc - float(mean_e)) < 5 * se + 1e-12, (trial, mc, float(mean_e))


def test_per_instance_counts(oracle_lib):
    g = from_edges(5, [0, 1, 2, 3], [1, 2, 3, 4], HALF)
    tot, per = oracle_lib.influence(g, 9, 8, [0], per_instance=True)
    assert per.sum() == tot and per.min() >= 1 and per.max() <= 5
