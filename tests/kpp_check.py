"""Validity check of a k-means++ seeding along its own trajectory.

k-means++ D^2 seeding (Arthur & Vassilvitskii, 2007) with the draws u given:
centre 0 = floor(u_0 N); centre j is the first index whose running sum of
D2 (squared distance to the nearest earlier centre) exceeds u_j W, W the
total.  Floating-point running sums depend on their order, so two correct
implementations can part where u_j W lies within rounding of a running sum.
This module checks a given centre sequence against the definition with
near-exact running sums of the same double-precision D2 (the oracle's
replay forms them in double-double arithmetic, relative error of order
N 2^-106, far below the rounding tolerated here):

  * every pick j has D2 > 0 (or W = 0 and it repeats centre j - 1);
  * S_{p-1} <= u_j W + tau and S_p >= u_j W - tau, where S are the running
    sums, p = centres[j], and tau bounds the rounding of the
    implementation's own running sums: a sum of m non-negative doubles, in
    any order, is within (m - 1) 2^-53 of its exact value relative to the
    total.

The oracle's flat pick on the same trajectory is returned beside it, so a
caller sees where, if anywhere, the two differ; each difference is a
certified tie (both picks valid).
"""
from fractions import Fraction

import numpy as np

import oracle

U53 = Fraction(1, 2 ** 53)


def _dd(pair):
    return Fraction(float(pair[0])) + Fraction(float(pair[1]))


def check_trajectory(X, u, centres, sum_terms):
    """Checks the seeding `centres` (K indices) of points X (N x 3) with draws
    u; `sum_terms` is the longest chain of additions in the
    implementation's running sums (its rounding budget).  Raises
    AssertionError on an invalid pick.  Returns the steps j where the
    oracle's flat pick on this trajectory differs from centres[j]."""
    X = np.ascontiguousarray(X, np.float64)
    N, K = X.shape[0], len(u)
    centres = np.asarray(centres, np.int64)
    assert centres.shape == (K,)
    flat, W2, before2, at2 = oracle.kmeanspp_replay(X, u, centres)
    assert centres[0] == flat[0], (centres[0], flat[0])
    ties = []
    budget = (sum_terms + 4) * U53
    for j in range(1, K):
        p = int(centres[j])
        W = _dd(W2[j])
        if W == 0:
            assert p == centres[j - 1], (j, p, "W = 0 must repeat the last centre")
            continue
        Slo, Shi = _dd(before2[j]), _dd(at2[j])
        assert Shi > Slo, (j, p, "a pick must have positive weight")
        t = Fraction(float(u[j])) * W
        tau = budget * W
        assert Slo <= t + tau and Shi >= t - tau, (
            j, p, float(Slo / W), float(Shi / W), float(u[j]),
            "pick outside the rounding of its running sum")
        if p != int(flat[j]):
            ties.append(j)
    return ties


def gpu_sum_terms(N):
    """Rounding budget of the GPU's running sums: chunks of 256 points
    (sequential), 16 chunk totals per thread (sequential) from an offset
    formed by a block scan of 1024 thread sums (6 shuffle levels, then 16
    wave totals in order), stages of 16,384 chunks in order, and inside the
    chosen chunk a block scan of its 256 terms (8 levels) from the chunk's
    running sum: at most 256 + 16 + 6 + 16 + 8 + ceil(N / 2^22) additions
    along a running sum, as many for the total W."""
    stages = -(-N // (256 * 16384))
    return 2 * (256 + 16 + 6 + 16 + 8 + stages)
