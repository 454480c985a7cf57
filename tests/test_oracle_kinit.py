"""Pins of the oracle's k-means++ seeding (the KInit step that precedes EM)
against an independent exact reference.

The reference below works in integer and rational arithmetic: points with
small integer coordinates make every squared distance an integer, the
draws are dyadic (m / 1024) so u * W is exact, and the running sum is one
flat int64 cumulative sum over all points.  The oracle forms the same flat
running sum in double precision; on these inputs both must pick exactly the
same centres and labels.  On general (non-integer) points the exact
reference sums the same double-precision squared distances as exact
integers (every double is an integer multiple of a common power of two).
With D^2 sampling written as "the first index whose running sum exceeds
u W", index i is drawn with probability D2_i / W (Arthur & Vassilvitskii,
2007).
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests.kpp_check import check_trajectory


def _exact_kmeanspp(Xi, K, u):
    """Integer / rational k-means++ with a flat running sum."""
    n = Xi.shape[0]

    def d2(c):
        d = Xi - Xi[c]
        return (d * d).sum(axis=1)

    c0 = min(int(Fraction(float(u[0])) * n), n - 1)
    cen = [c0]
    D = d2(c0)
    for j in range(1, K):
        W = int(D.sum())
        if W == 0:
            pick = cen[-1]
        else:
            t = Fraction(float(u[j])) * W
            cs = np.cumsum(D)
            # first i with cs[i] > t; cs is integer, so cs > t <=> cs > floor(t)
            pick = int(np.searchsorted(cs, int(t), side="right"))
        cen.append(pick)
        D = np.minimum(D, d2(pick))
    dist = np.stack([d2(c) for c in cen], axis=1)
    return np.array(cen, dtype=np.int64), np.argmin(dist, axis=1).astype(np.int32)


def _int_cloud(seed, n, hi=40):
    return np.random.default_rng(seed).integers(0, hi, (n, 3)).astype(np.int64)


def _dyadic(seed, K):
    return np.random.default_rng(seed).integers(0, 1024, K) / 1024.0


@pytest.mark.parametrize("n,K", [(1, 1), (5, 3), (257, 17), (1000, 40),
                                 (20000, 12), (16385, 5)])
def test_kmeanspp_matches_exact_reference(n, K):
    Xi = _int_cloud(n + K, n)
    u = _dyadic(n * 7 + K, K)
    cen, lab = oracle.kmeanspp(Xi.astype(np.float64), K, u)
    rc, rl = _exact_kmeanspp(Xi, K, u)
    np.testing.assert_array_equal(cen, rc)
    np.testing.assert_array_equal(lab, rl)


def test_kmeanspp_draw_zero_and_near_one():
    """u = 0 picks the first point with positive weight; u just below 1
    (u W rounds up to W in double) picks the last one."""
    Xi = _int_cloud(3, 3000)
    Xi[:10] = Xi[0]                       # points 1..9 coincide with point 0
    u = np.array([0.0, 0.0, 1.0 - 2.0 ** -53, 0.5, 1.0 - 2.0 ** -53])
    cen, lab = oracle.kmeanspp(Xi.astype(np.float64), 5, u)
    rc, rl = _exact_kmeanspp(Xi, 5, u)
    np.testing.assert_array_equal(cen, rc)
    np.testing.assert_array_equal(lab, rl)
    assert cen[0] == 0 and cen[1] == 10   # first point off centre 0


def test_kmeanspp_all_points_equal():
    """W = 0 after the first centre: every later centre repeats it and
    every label is 0."""
    X = np.tile(np.array([[1.5, -2.0, 3.25]]), (300, 1))
    cen, lab = oracle.kmeanspp(X, 4, np.array([0.7, 0.1, 0.2, 0.3]))
    assert list(cen) == [210, 210, 210, 210]
    assert not lab.any()


def test_kmeanspp_label_ties_go_to_the_lowest_index():
    X = np.array([[0.0, 0, 0], [2.0, 0, 0], [1.0, 0, 0], [1.0, 5, 0]])
    # D2 from point 0: [0, 4, 1, 26], W = 31; u = 0.1 -> t = 3.1 -> point 1
    cen, lab = oracle.kmeanspp(X, 2, np.array([0.0, 0.1]))
    rc, rl = _exact_kmeanspp(X.astype(np.int64), 2, np.array([0.0, 0.1]))
    np.testing.assert_array_equal(cen, rc)
    np.testing.assert_array_equal(lab, rl)
    assert list(cen) == [0, 1]
    assert list(lab) == [0, 1, 0, 0]      # points 2 and 3 are equidistant


def _exact_ints(D):
    """The doubles D as exact integers, all scaled by one power of two."""
    parts = [float(v).as_integer_ratio() for v in D]
    den = max(q for _, q in parts)
    return [n * (den // q) for n, q in parts]


def _exact_general_kmeanspp(X, K, u):
    """Flat running sums in exact arithmetic of the double-precision D2."""
    N = X.shape[0]

    def d2(c):
        d = X - X[c]
        return (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]

    c = [min(int(u[0] * N), N - 1)]
    D = d2(c[0])
    for j in range(1, K):
        Di = _exact_ints(D)
        S = list(itertools.accumulate(Di))
        W = S[-1]
        un, ud = float(u[j]).as_integer_ratio()
        # first i with S_i > u W  <=>  S_i ud > un W
        lim = un * W
        i = next(i for i, s_ in enumerate(S) if s_ * ud > lim)
        c.append(i)
        D = np.minimum(D, d2(i))
    return np.array(c, dtype=np.int64)


@pytest.mark.parametrize("n,K,seed", [(700, 6, 11), (40000, 10, 12), (20011, 25, 13)])
def test_kmeanspp_general_points_match_exact_running_sum(n, K, seed):
    """Non-integer coordinates over many 256-point chunks and several
    64-chunk groups: the oracle's double-precision flat running sum picks
    the same centres as the exact running sum of the same squared
    distances, and its labels are the nearest centres."""
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 3, (n, 3)).astype(np.float32).astype(np.float64)
    X[: n // 3] *= 0.01                    # a dense core: D2 over many scales
    u = rng.random(K)
    cen, lab = oracle.kmeanspp(X, K, u)
    np.testing.assert_array_equal(cen, _exact_general_kmeanspp(X, K, u))
    np.testing.assert_array_equal(lab, oracle.nearest(X, cen))
    d = np.stack([((X - X[c]) ** 2).sum(axis=1) for c in cen], axis=1)
    assert (d[np.arange(n), lab] <= d.min(axis=1) * (1 + 1e-12)).all()


def test_trajectory_check_accepts_the_oracle_and_rejects_a_wrong_pick():
    """The validity check used on the GPU's seeding: the oracle's own picks
    pass with no tie; moving one pick to a neighbouring index, or to a
    point already chosen (weight 0), fails."""
    rng = np.random.default_rng(21)
    X = rng.normal(0, 2, (30000, 3)).astype(np.float32).astype(np.float64)
    K = 20
    u = rng.random(K)
    cen, _ = oracle.kmeanspp(X, K, u)
    assert check_trajectory(X, u, cen, sum_terms=30000) == []
    for j, bad in ((7, cen[7] + 1), (7, cen[7] - 1), (12, cen[3])):
        wrong = cen.copy()
        wrong[j] = bad
        with pytest.raises(AssertionError):
            check_trajectory(X, u, wrong, sum_terms=30000)


def test_nearest_labels_ties_and_argument_checks():
    X = np.array([[0.0, 0, 0], [2.0, 0, 0], [1.0, 0, 0], [5.0, 0, 0]])
    assert list(oracle.nearest(X, [0, 1])) == [0, 1, 0, 1]
    assert list(oracle.nearest(X, [1, 0])) == [1, 0, 0, 0]
    with pytest.raises(oracle.OracleError):
        oracle.nearest(X, [0, 4])


@pytest.mark.parametrize("bad", ["k_gt_n", "u_one", "u_neg", "nan"])
def test_kmeanspp_rejects_bad_input(bad):
    X = np.random.default_rng(0).random((10, 3))
    u = np.full(3, 0.5)
    K = 3
    if bad == "k_gt_n":
        K, u = 11, np.full(11, 0.5)
    elif bad == "u_one":
        u[1] = 1.0
    elif bad == "u_neg":
        u[2] = -0.1
    else:
        X[4, 1] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.kmeanspp(X, K, u)
