"""Pins of the mean-shift oracle (oracle/gbms.py) against things other than
itself:

* scikit-learn's MeanShift (flat kernel) as a black box, started from the
  oracle's seeds: the same modes in the same order, and scikit-learn's own
  binned seeds against the oracle's (float32 there);
* clouds whose modes are known: identical points (the mode is the point,
  its weight the multiplicity), well-separated Gaussian blobs (one mode per
  blob, at the blob's mean within the sampling error), two groups closer
  than the bandwidth (one mode at the pooled mean);
* the merge rule on its own (a heavier mode removes every lighter one
  within h; ties in weight go to the lexicographically larger mode).
"""
import warnings

import numpy as np
import pytest

from oracle import gbms as og


def _blobs(seed, k=4, n=300, d=3, sep=6.0, sigma=0.25):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-1, 1, (k, d)) * sep * 2
    # keep the centres apart
    while True:
        dd = np.linalg.norm(centres[:, None] - centres[None], axis=-1) + np.eye(k) * 1e9
        if dd.min() > sep:
            break
        centres = rng.uniform(-1, 1, (k, d)) * sep * 2
    X = np.concatenate([c + sigma * rng.standard_normal((n, d)) for c in centres])
    return X.astype(np.float32).astype(np.float64), centres


@pytest.mark.parametrize("d", [3, 4])
def test_modes_match_sklearn_meanshift_from_the_same_seeds(d):
    from sklearn.cluster import MeanShift, get_bin_seeds
    X, _ = _blobs(1, k=5, n=200, d=d)
    h = 1.2
    modes, w, _ = og.gbms(X, h)
    seeds = og.bin_seeds(X, h)
    ms = MeanShift(bandwidth=h, seeds=seeds, max_iter=300)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        ms.fit(X)
    np.testing.assert_allclose(modes, ms.cluster_centers_, rtol=0, atol=1e-12)
    sk = get_bin_seeds(X, h, min_bin_freq=1)
    a = np.array(sorted(map(tuple, np.asarray(sk, np.float64))))
    b = np.array(sorted(map(tuple, seeds)))
    np.testing.assert_allclose(a, b, rtol=1e-6, atol=1e-6)


def test_identical_points_are_their_own_modes():
    X = np.array([[0.0, 0, 0]] * 5 + [[10.0, 0, 0]] * 3 + [[0.0, 20, 0]] * 5)
    modes, w, _ = og.gbms(X, 1.0)
    # equal weights 5 and 5: the lexicographically larger mode comes first
    np.testing.assert_array_equal(modes, [[0.0, 20, 0], [0.0, 0, 0], [10.0, 0, 0]])
    np.testing.assert_array_equal(w, [5, 5, 3])


@pytest.mark.parametrize("seed,d", [(2, 3), (3, 4), (4, 3)])
def test_one_mode_per_separated_blob(seed, d):
    X, centres = _blobs(seed, k=4, n=400, d=d, sep=8.0, sigma=0.3)
    modes, w, _ = og.gbms(X, 1.5)
    assert modes.shape == (4, d)
    for c in centres:
        dist = np.linalg.norm(modes - c, axis=1)
        assert dist.min() <= 0.1, dist.min()
    assert w.sum() <= X.shape[0] and w.min() > 300


def test_groups_closer_than_the_bandwidth_merge():
    rng = np.random.default_rng(7)
    a = np.array([0.0, 0, 0]) + 0.02 * rng.standard_normal((100, 3))
    b = np.array([0.6, 0, 0]) + 0.02 * rng.standard_normal((100, 3))
    X = np.concatenate([a, b])
    modes, w, _ = og.gbms(X, 1.0)
    assert modes.shape == (1, 3)
    np.testing.assert_allclose(modes[0], X.mean(axis=0), atol=1e-12)
    assert w[0] == 200


def test_merge_rule():
    """Modes 0.5 apart with h = 1: the heavier one stays; a third mode 3
    away stays as well; weight ties go to the larger coordinates."""
    X = np.concatenate([np.zeros((6, 3)), np.tile([[0.5, 0, 0]], (4, 1)),
                        np.tile([[3.0, 0, 0]], (2, 1))])
    # with h = 0.3 every group is its own mode; merging at h = 1 is what the
    # oracle's merge step does to that list
    modes, w, (all_m, all_w) = og.gbms(X, 0.3)
    assert modes.shape == (3, 3)
    h = 1.0
    keep = np.ones(len(all_w), bool)
    for i in range(len(all_w)):
        if keep[i]:
            far = np.linalg.norm(all_m - all_m[i], axis=1) > h
            far[: i + 1] = True
            keep &= far
    np.testing.assert_array_equal(all_m[keep], [[0.0, 0, 0], [3.0, 0, 0]])
    X2 = np.array([[1.0, 0, 0]] * 3 + [[2.0, 0, 0]] * 3)
    modes2, w2, _ = og.gbms(X2, 0.5)
    np.testing.assert_array_equal(modes2, [[2.0, 0, 0], [1.0, 0, 0]])


def test_merge_chain_and_ties():
    """A removed mode removes nothing: in the chain A (w 5) - B (w 4) - C
    (w 3), 0.8 apart with h = 1, B goes (A is within h) and C stays (only B
    is within h of it), which a rule 'drop a mode with any heavier mode
    within h' would get wrong.  Identical (weight, mode) pairs keep the
    first seed."""
    modes = np.array([[1.6, 0, 0], [0.0, 0, 0], [0.8, 0, 0]])
    w = np.array([3, 5, 4])
    mask, order = og.merge(modes, w, 1.0)
    np.testing.assert_array_equal(order, [1, 2, 0])
    np.testing.assert_array_equal(mask, [True, True, False])
    dup = np.array([[2.0, 1, 1], [2.0, 1, 1], [2.0, 1, 1]])
    mask, order = og.merge(dup, np.array([7, 7, 7]), 0.5)
    np.testing.assert_array_equal(order, [0, 1, 2])
    np.testing.assert_array_equal(mask, [True, False, False])
    # exactly h apart: removed (the test is <=)
    mask, _ = og.merge(np.array([[0.0, 0, 0], [0.5, 0, 0]]), np.array([2, 1]), 0.5)
    np.testing.assert_array_equal(mask, [True, False])
