"""Pins for the oracle's SKIM (Section 4, Algorithm 1).

* Correctness statement (Section 4.1.1): the gains I_1..I_s sum to the exact
  influence of the seed prefix, for every prefix (integer pair counts).
* With k above every |R_u| no sketch fills, every rank is processed and each
  seed comes from the exhaustion rule, which is exact greedy: brute-force
  greedy (max marginal gain, smallest id on ties) must match seed for seed.
* The first seed is the node whose sketch fills first, i.e. the smallest
  threshold rank tau among full sketches (Section 4: it has the maximum
  estimated influence).
* Seeds are distinct; running to s = n covers every pair.
"""
import numpy as np

from workloads import from_edges
from workloads.configs import make_config, make_graph
from brute import greedy_exact, random_small_graph


def _check_prefix_sums(oracle_lib, g, seed, ell, seeds, gains):
    tot = 0
    for j in range(len(seeds)):
        tot += int(gains[j])
        assert tot == oracle_lib.influence(g, seed, ell, seeds[:j + 1])


def test_gains_sum_to_influence_tiny_config(oracle_lib):
    cfg = make_config("served-skim")
    g = make_graph(cfg)
    seeds, gains, cnt = oracle_lib.skim(g, cfg["seed"], cfg["ell"], cfg["k"], 60)
    assert len(set(seeds.tolist())) == 60
    _check_prefix_sums(oracle_lib, g, cfg["seed"], cfg["ell"], seeds, gains)
    assert cnt["covered"] == int(gains.sum())


def test_first_seed_is_smallest_threshold(oracle_lib):
    rng = np.random.default_rng(5)
    for trial in range(5):
        n = 60
        src, dst, thr = random_small_graph(rng, n, 200, [0xFFFFFFFF // 4, 0xFFFFFFFF // 2])
        g = from_edges(n, src, dst, thr)
        ell, k, seed = 8, 6, 100 + trial
        ranks, size, _ = oracle_lib.build_alg2(g, seed, ell, k)
        full = np.where(size == k)[0]
        tau = ranks[full, k - 1]
        want = int(full[np.argmin(tau)])  # ranks are distinct: no tie
        seeds, gains, _ = oracle_lib.skim(g, seed, ell, k, 1)
        assert int(seeds[0]) == want
        assert int(gains[0]) == oracle_lib.influence(g, seed, ell, [want])


def test_exhaustion_is_exact_greedy(oracle_lib):
    rng = np.random.default_rng(6)
    for trial in range(6):
        n = int(rng.integers(5, 25))
        src, dst, thr = random_small_graph(rng, n, int(rng.integers(0, 3 * n)),
                                           [0xFFFFFFFF // 2, 0xFFFFFFFF])
        g = from_edges(n, src, dst, thr)
        ell, seed = 4, 300 + trial
        k = n * ell + 1  # above every |R_u|
        s = n
        seeds, gains, cnt = oracle_lib.skim(g, seed, ell, k, s)
        gs, gg = greedy_exact(g, seed, ell, s, oracle_lib)
        assert seeds.tolist() == gs and gains.tolist() == gg
        assert cnt["fallback"] == s
        assert int(gains.sum()) == n * ell  # a full permutation covers everything
        assert (np.diff(gains.astype(np.int64)) <= 0).all()  # greedy gains never grow


def test_full_permutation_properties(oracle_lib):
    rng = np.random.default_rng(8)
    n = 40
    src, dst, thr = random_small_graph(rng, n, 120, [0xFFFFFFFF // 3])
    g = from_edges(n, src, dst, thr)
    seeds, gains, _ = oracle_lib.skim(g, 5, 16, 8, n)
    assert sorted(seeds.tolist()) == list(range(n))
    assert int(gains.sum()) == n * 16
    _check_prefix_sums(oracle_lib, g, 5, 16, seeds, gains)
