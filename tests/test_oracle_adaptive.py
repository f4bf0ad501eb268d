"""Pins for the oracle's adaptive error estimate (Section 4, adaptive error
estimation, eq. (chernoff)) and for SKIM's per-seed records behind it.

* eq. (chernoff) is a true bound on the lower tail of a sum of independent
  Bernoulli trials: it must lie above the exact Poisson and binomial tails
  (scipy), equal P[Poisson(mu) = 0] = e^-mu at z = 0, and have the exact large
  deviations exponent mu (a - 1 - a ln a) of the Poisson lower tail.
* The convolution: one iteration gives its own survival function; two give
  what a brute-force double sum over their distributions gives; exhaustion
  records (D = 0) change nothing; tails fall with j and only grow as
  iterations are added.
* The records tau and k' of the oracle's SKIM equal their definitions,
  recomputed from scratch per iteration on tiny graphs: tau is the smallest
  k-th uncovered rank over unselected nodes, k' the largest count of
  uncovered ranks below tau among the other unselected nodes.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import logsumexp

from oracle import adaptive as ad
from workloads import from_edges
from workloads.configs import make_config, make_graph
from brute import live_adjacency, random_small_graph, reach


# ------------------------------------------------------------ eq. (chernoff)

@pytest.mark.parametrize("mu", [0.5, 3.0, 20.0, 150.0, 900.0])
def test_chernoff_bounds_exact_lower_tails(mu):
    for a in (0.0, 0.1, 0.35, 0.6, 0.85, 0.97, 1.0, 1.3):
        z = a * mu
        b = ad.chernoff_bound(mu, z)
        assert 0.0 <= b <= 1.0
        if z >= mu:
            assert b == 1.0
            continue
        zi = math.ceil(z) - 1  # Z < z  <=>  Z <= ceil(z) - 1 for integer Z
        pois = stats.poisson.cdf(zi, mu) if zi >= 0 else 0.0
        assert b >= pois * (1 - 1e-12)
        N = int(math.ceil(4 * mu)) + 1
        binom = stats.binom.cdf(zi, N, mu / N) if zi >= 0 else 0.0
        assert b >= binom * (1 - 1e-12)


@pytest.mark.parametrize("mu", [0.25, 1.0, 7.5, 60.0, 700.0])
def test_chernoff_at_zero_is_poisson_zero(mu):
    assert ad.chernoff_bound(mu, 0.0) == pytest.approx(stats.poisson.pmf(0, mu), rel=1e-12)


@pytest.mark.parametrize("a", [0.2, 0.5, 0.8])
def test_chernoff_exponent_is_the_large_deviation_rate(a):
    mu = 20000.0
    z = a * mu
    # log of the bound, from the bound itself (avoid underflow by scaling mu)
    lb = math.log(ad.chernoff_bound(mu / 1000.0, z / 1000.0)) * 1000.0
    assert lb == pytest.approx(mu * (a - 1 - a * math.log(a)), rel=1e-9)
    lp = float(logsumexp(stats.poisson.logpmf(np.arange(math.ceil(z)), mu)))
    # the bound is loose only by a factor polynomial in mu, never by e^(c mu)
    assert 0.0 <= lb - lp <= math.log(2 * math.pi * mu)


# ----------------------------------------------------------- the convolution

def _recs(rng, s, scan_frac=0.8):
    tau = np.where(rng.random(s) < scan_frac,
                   rng.integers(1 << 56, 1 << 62, size=s, dtype=np.uint64),
                   np.uint64(ad.NONE)).astype(np.uint64)
    gain = rng.integers(20, 400, size=s).astype(np.uint64)
    second = rng.integers(0, 40, size=s).astype(np.uint32)
    return tau, second, gain


def test_single_iteration_tail_is_its_survival():
    tau = [1 << 61]
    for k2 in (0, 5, 31):
        tail = ad.discrepancy_tail(tau, [k2], [300], 64, 0.5)
        h = 0.5 * 300 / 64
        S = ad.iteration_survival(tau[0], k2, 300, h, 64)
        assert np.allclose(tail, S, rtol=0, atol=1e-15)
        if k2 == 0:  # closed form: exp(-tau Delta (1 + eps))
            t = ad.rho(tau[0])
            for j in range(1, 65):
                want = math.exp(-t * 300 * (1 + (j - 1) * h / 300))
                assert tail[j] == pytest.approx(want, rel=1e-12)


def test_two_iterations_match_brute_force_sum():
    rng = np.random.default_rng(3)
    for trial in range(4):
        tau, second, gain = _recs(rng, 2, scan_frac=1.0)
        bins = int(rng.integers(5, 40))
        tail = ad.discrepancy_tail(tau, second, gain, bins, 0.3)
        h = 0.3 * float(gain.sum()) / bins
        pm = []
        for t, k2, d in zip(tau, second, gain):
            S = ad.iteration_survival(t, k2, d, h, bins)
            pm.append([S[j] - (S[j + 1] if j < bins else 0.0) for j in range(bins + 1)])
        for j in range(bins + 1):
            want = sum(pm[0][a] * pm[1][b] for a in range(bins + 1) for b in range(bins + 1)
                       if min(a + b, bins) >= j)
            assert tail[j] == pytest.approx(want, rel=1e-12, abs=1e-15)


def test_tail_properties():
    rng = np.random.default_rng(4)
    tau, second, gain = _recs(rng, 30)
    bins = 200
    tail = ad.discrepancy_tail(tau, second, gain, bins, 0.4)
    assert tail[0] == pytest.approx(1.0, abs=1e-12)
    assert np.all(np.diff(tail) <= 1e-15) and np.all(tail >= -1e-15)
    # adding iterations never lowers the bound (the discrepancies are >= 0);
    # the grid step is held fixed by rescaling max_rel_error
    prev = None
    I = float(gain.sum())
    for s in range(1, 31):
        rel = 0.4 * I / float(gain[:s].sum())
        t = ad.discrepancy_tail(tau[:s], second[:s], gain[:s], bins, rel)
        if prev is not None:
            assert np.all(t >= prev - 1e-12)
        prev = t


def test_exhaustion_records_change_nothing():
    rng = np.random.default_rng(5)
    tau, second, gain = _recs(rng, 12, scan_frac=1.0)
    base = ad.discrepancy_tail(tau, second, gain, 100, 0.2)
    ex_tau = np.concatenate([tau, np.full(5, ad.NONE, dtype=np.uint64)])
    ex_sec = np.concatenate([second, np.full(5, 7, dtype=np.uint32)])
    ex_gain = np.concatenate([gain, np.zeros(5, dtype=np.uint64)])  # keeps I unchanged
    assert np.array_equal(ad.discrepancy_tail(ex_tau, ex_sec, ex_gain, 100, 0.2), base)
    only = ad.discrepancy_tail([ad.NONE] * 3, [4] * 3, [9, 5, 1], 50, 0.3)
    assert only[0] == 1.0 and not np.any(only[1:])
    assert np.array_equal(ad.discrepancy_tail([], [], [], 8, 0.1), np.eye(1, 9)[0])
    # a filled-sketch record with no gain carries no bound at all
    assert np.all(ad.discrepancy_tail([1 << 60, ad.NONE], [3, 0], [0, 5], 8, 0.1) == 1.0)


# --------------------------------------------------- SKIM's per-seed records

def _records_from_scratch(g, seed, ell, k, seeds, oracle):
    adj = live_adjacency(g, seed, ell, oracle)
    sets = [set((v, i) for i in range(ell) for v in reach(adj[i], [u])) for u in range(g.n)]
    rank = {(v, i): oracle.rank(seed, v, i) for v in range(g.n) for i in range(ell)}
    covered, chosen = set(), set()
    taus, seconds = [], []
    for x in seeds:
        x = int(x)
        unc = {u: sorted(rank[p] for p in sets[u] - covered) for u in range(g.n) if u not in chosen}
        kth = {u: r[k - 1] for u, r in unc.items() if len(r) >= k}
        if kth:
            tau = min(kth.values())
            assert x == min(u for u, r in kth.items() if r == tau)
            second = max([sum(1 for r in unc[u] if r < tau) for u in unc if u != x] or [0])
        else:
            tau = ad.NONE
            best = max(len(r) for r in unc.values())
            assert x == min(u for u, r in unc.items() if len(r) == best)
            second = max([len(unc[u]) for u in unc if u != x] or [0])
        taus.append(tau)
        seconds.append(second)
        covered |= sets[x]
        chosen.add(x)
    return taus, seconds


def test_skim_records_match_their_definition(oracle_lib):
    rng = np.random.default_rng(11)
    for trial in range(6):
        n = int(rng.integers(8, 22))
        src, dst, thr = random_small_graph(rng, n, int(rng.integers(n, 4 * n)),
                                           [0xFFFFFFFF // 3, 0xFFFFFFFF // 2])
        g = from_edges(n, src, dst, thr)
        ell, k, seed = int(rng.integers(2, 6)), int(rng.integers(2, 6)), 500 + trial
        s = n  # runs on into the exhaustion rule
        seeds, gains, tau, second, _ = oracle_lib.skim(g, seed, ell, k, s, records=True)
        want_tau, want_second = _records_from_scratch(g, seed, ell, k, seeds, oracle_lib)
        assert [int(t) for t in tau] == want_tau
        assert [int(x) for x in second] == want_second
        scan = np.array([int(t) != ad.NONE for t in tau])
        assert np.all(second[scan] <= k - 1)


def test_skim_records_on_the_served_config(oracle_lib):
    cfg = make_config("served-skim")
    g = make_graph(cfg)
    seeds, gains, tau, second, cnt = oracle_lib.skim(g, cfg["seed"], cfg["ell"], cfg["k"], 200,
                                                      records=True)
    assert cnt["fallback"] == 0 and np.all(tau != ad.NONE)
    assert np.all(np.diff(tau.astype(object)) > 0)  # thresholds rise seed after seed
    assert np.all(second <= cfg["k"] - 1)
    plain_seeds, plain_gains, _ = oracle_lib.skim(g, cfg["seed"], cfg["ell"], cfg["k"], 200)
    assert np.array_equal(plain_seeds, seeds) and np.array_equal(plain_gains, gains)
    tail = ad.discrepancy_tail(tau, second, gains, 256, 0.5)
    assert tail[0] == pytest.approx(1.0) and tail[-1] < tail[0]
