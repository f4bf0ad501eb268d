"""Pins for the oracle's randomness: SplitMix64 ranks and live-edge coins.

The paper draws an independent U[0,1] rank per node-instance pair (Section 3)
and a biased coin per edge and instance (binary IC, Section 1).  The oracle
realises both with SplitMix64; these tests pin that generator to its published
outputs and to properties fixed by mathematics, not to itself.
"""
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
M64 = (1 << 64) - 1


def _golden_splitmix():
    vals = []
    with open(os.path.join(HERE, "golden", "splitmix64_seed0.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                vals.append(int(line, 16))
    return vals


def _golden_gamma():
    """The odd integer nearest 2^64 / phi (the golden-ratio increment)."""
    getcontext().prec = 60
    phi = (1 + Decimal(5).sqrt()) / 2
    x = Decimal(2 ** 64) / phi
    g = int(x)
    return g if g % 2 == 1 else g + 1


def _unmix(z):
    """Inverse of the variant-13 finaliser (xor-shifts and odd multipliers)."""
    def unxorshift(y, s):
        x = y
        for _ in range(64 // s + 1):
            x = y ^ (x >> s)
        return x & M64

    z = unxorshift(z, 31)
    z = (z * pow(0x94D049BB133111EB, -1, 1 << 64)) & M64
    z = unxorshift(z, 27)
    z = (z * pow(0xBF58476D1CE4E5B9, -1, 1 << 64)) & M64
    z = unxorshift(z, 30)
    return z


def test_splitmix_published_outputs(oracle_lib):
    want = _golden_splitmix()
    got = [oracle_lib.sm64(0, c) for c in range(len(want))]
    assert got == want


def test_splitmix_increment_is_golden_gamma(oracle_lib):
    # mix64 is a bijection; undoing it must give the counter times the odd
    # increment derived from the golden ratio (nothing else is added).
    gamma = _golden_gamma()
    assert gamma == 0x9E3779B97F4A7C15
    for seed in (0, 1, 12345, M64):
        for c in (0, 1, 2, 63, 1 << 40):
            assert _unmix(oracle_lib.sm64(seed, c)) == (seed + (c + 1) * gamma) & M64


def test_ranks_are_distinct_and_uniform(oracle_lib):
    n, ell = 20000, 64
    r = oracle_lib.ranks(1, n, ell).reshape(-1)
    assert np.unique(r).size == r.size
    # rank of pair (v, i) is stream output 64 v + i
    assert int(r[5 * ell + 3]) == oracle_lib.sm64(1, 64 * 5 + 3)
    assert oracle_lib.rank(1, 5, 3) == oracle_lib.sm64(1, 64 * 5 + 3)
    # uniformity of the top 4 bits: chi-square with 15 dof, loose bound
    top = (r >> np.uint64(60)).astype(np.int64)
    cnt = np.bincount(top, minlength=16)
    exp = r.size / 16
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert chi2 < 60


def test_ranks_do_not_depend_on_ell(oracle_lib):
    # r(v, i) = SM(seed, 64 v + i): instances are nested across l
    a = oracle_lib.ranks(7, 50, 16)
    b = oracle_lib.ranks(7, 50, 64)
    assert np.array_equal(a, b[:, :16])


def test_live_extremes(oracle_lib):
    rng = np.random.default_rng(0)
    u = rng.integers(0, 1000, 5000)
    v = rng.integers(0, 1000, 5000)
    inst = rng.integers(0, 64, 5000)
    assert oracle_lib.live_batch(3, 1000, u, v, inst, 0xFFFFFFFF).all()
    # thr = 0 fires with probability 2^-32 per draw
    assert not oracle_lib.live_batch(3, 1000, u, v, inst, 0).any()


@pytest.mark.parametrize("denom", [2, 20, 100, 1000])
def test_live_rate_within_5_sigma(oracle_lib, denom):
    thr = 0xFFFFFFFF // denom
    p = (thr + 1) / 2 ** 32
    n = 3000
    N = 400_000
    rng = np.random.default_rng(denom)
    u = rng.integers(0, n, N)
    v = rng.integers(0, n, N)
    inst = rng.integers(0, 64, N)
    hits = oracle_lib.live_batch(11, n, u, v, inst, thr).sum()
    sigma = np.sqrt(N * p * (1 - p))
    assert abs(hits - N * p) < 5 * sigma


def test_live_instances_independent(oracle_lib):
    # the two halves of one 64-bit output serve instances 2j and 2j+1:
    # their coins must be uncorrelated, as must different edges
    thr = 0xFFFFFFFF // 2
    n = 5000
    N = 200_000
    rng = np.random.default_rng(5)
    u = rng.integers(0, n, N)
    v = rng.integers(0, n, N)
    j = rng.integers(0, 32, N)
    a = oracle_lib.live_batch(2, n, u, v, 2 * j, thr).astype(float)
    b = oracle_lib.live_batch(2, n, u, v, 2 * j + 1, thr).astype(float)
    c = np.corrcoef(a, b)[0, 1]
    assert abs(c) < 5 / np.sqrt(N)
    # the coin depends on the seed
    d = oracle_lib.live_batch(3, n, u, v, 2 * j, thr).astype(float)
    assert abs(np.corrcoef(a, d)[0, 1]) < 5 / np.sqrt(N)


def test_rank_inversion_recovers_pairs(oracle_lib):
    """The test helper that maps a rank back to its pair inverts the oracle's
    rank function exactly (used to check full-size sketches pair by pair)."""
    from brute import rank_to_pair
    rng = np.random.default_rng(11)
    for seed in (0, 1, 0xDEADBEEFCAFEF00D):
        v = rng.integers(0, 1 << 25, 2000)
        i = rng.integers(0, 64, 2000)
        r = np.array([oracle_lib.rank(seed, int(a), int(b)) for a, b in zip(v, i)], dtype=np.uint64)
        p = rank_to_pair(r, seed)
        assert np.array_equal(p, (v * 64 + i).astype(np.uint64))
