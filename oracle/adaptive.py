"""Adaptive error estimate of a SKIM run (Section 4, "Adaptive Error
Estimation", eq. (chernoff)), written plainly in numpy / fp64.

TEST INFRASTRUCTURE ONLY: the reference the HIP library's
``skim_discrepancy_tail`` is checked against.  Only the tests, the smoke check
and the bench's CPU-baseline leg may import it.  It shares no code with the
HIP path.

What is computed.  Iteration s of SKIM selects a seed of exact marginal gain
Delta_s (node-instance pairs).  Its discrepancy D_s is the gap between the
largest marginal gain of any node and Delta_s.  If the true maximum exceeded
Delta_s (1 + eps), that node's expected sketch size at the seed's threshold
rank tau_s would be at least mu = tau_s Delta_s (1 + eps), yet its sketch holds
at most k'_s ranks (the second largest sketch).  eq. (chernoff) with Z = k'_s
and nu = 1 - k'_s / mu bounds the probability of that event:

    P[D_s > eps Delta_s] <= B_s(eps) = (exp(-nu) / (1 - nu)^(1 - nu))^mu,

and B_s = 1 where mu <= k'_s (nothing is claimed).  The bound on the sum of
the discrepancies is the convolution, iteration after iteration, of the
per-iteration distributions (Section 4: "take a convolution, after each
iteration").

Readings (the paper gives the formula, not the discretisation):
  * tau_s is the real reading rho(T) = ((T >> 11) + 1) 2^-53 of the 64-bit rank
    T of the pair that filled the seed's sketch; Delta_s and k'_s count pairs.
  * A seed chosen by the exhaustion rule (tau = 2^64 - 1) has D_s = 0: with
    every rank processed the sizes are the exact residual gains.
  * A filled-sketch record with Delta_s = 0 carries no bound (B_s = 1).
  * Discrepancies are measured on a grid of step h = max_rel_error * I / bins
    pairs, I = sum_s Delta_s (the seed set's influence times l).  Each D_s is
    replaced by h * ceil(D_s / h), which is never smaller, so
        P[ceil(D_s/h) >= j] = P[D_s > (j-1) h] <= B_s((j-1) h / Delta_s)
    for j >= 1; everything at or beyond bins * h is kept in the last cell (so
    the cap only makes the bound more conservative).
  * Output: tail[j] = an upper bound on P[sum_s D_s >= j h], j = 0..bins.
  * With no records, or I = 0, tail = (1, 0, ..., 0).
"""
from __future__ import annotations

import math

import numpy as np

NONE = 0xFFFFFFFFFFFFFFFF


def rho(T: int) -> float:
    """Real reading of a 64-bit rank (Section 3: U[0,1] ranks)."""
    return float((int(T) >> 11) + 1) * 2.0 ** -53


def chernoff_bound(mu: float, z: float) -> float:
    """eq. (chernoff): bound on P[Z < z] for a sum Z of independent Bernoulli
    trials of mean mu, with z = (1 - nu) mu; 1 where z >= mu."""
    if z >= mu:
        return 1.0
    nu = 1.0 - z / mu
    one_minus = 1.0 - nu
    base = math.exp(-nu) / (one_minus ** one_minus)  # 0^0 = 1 at z = 0
    return base ** mu


def iteration_survival(tau: int, second: int, gain: int, h: float, bins: int) -> np.ndarray:
    """S[j] = bound on P[ceil(D_s / h) >= j], j = 0..bins (S[0] = 1)."""
    S = np.zeros(bins + 1)
    S[0] = 1.0
    if int(tau) == NONE:
        return S                      # exhaustion: exact choice, D_s = 0
    if int(gain) == 0:
        S[:] = 1.0                    # no bound
        return S
    t = rho(tau)
    for j in range(1, bins + 1):
        eps = (j - 1) * h / float(gain)
        mu = t * float(gain) * (1.0 + eps)
        S[j] = min(1.0, chernoff_bound(mu, float(second)))
    return S


def discrepancy_tail(tau, second, gain, bins: int, max_rel_error: float) -> np.ndarray:
    """tail[j] >= P[sum of discrepancies >= j * max_rel_error * I / bins]."""
    tau = [int(x) for x in tau]
    second = [int(x) for x in second]
    gain = [int(x) for x in gain]
    assert bins >= 1 and max_rel_error > 0
    total = sum(gain)
    dist = np.zeros(bins + 1)
    dist[0] = 1.0                     # empty sum: 0 with certainty
    if total == 0:
        return dist.copy()
    h = max_rel_error * float(total) / float(bins)
    for t, k2, d in zip(tau, second, gain):
        S = iteration_survival(t, k2, d, h, bins)
        pmf = S - np.append(S[1:], 0.0)
        full = np.convolve(dist, pmf)   # distribution of the (uncapped) sum
        dist = full[:bins + 1].copy()
        dist[bins] += full[bins + 1:].sum()
    return np.cumsum(dist[::-1])[::-1]
