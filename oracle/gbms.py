"""FP64 oracle of the component-count estimate that precedes k-means
seeding and EM: mean shift with a flat kernel and binned seeds.

TEST INFRASTRUCTURE ONLY.  The test suite and the benchmark's CPU-baseline
leg are the only callers; nothing in the HIP library imports or runs this
module, and it uses nothing of the HIP library.  Plain numpy, double
precision, one seed at a time, brute-force radius queries.

What is computed (the paper, Sec. V "Gaussian Blurring Mean Shift" and the
information-flow figure: a bandwidth and the point cloud give the number
of components K through mean shift, binned seeds after Comaniciu & Meer,
radius-neighbour averages, termination by an iteration cap or a vanishing
shift):

  seeds     the centres b h of the bins b = round(x / h) (round half to
            even, per coordinate) that hold at least one point, h the
            bandwidth;
  shift     from a seed s, repeatedly: W = the points within distance h
            of s (squared distance <= h^2), s <- mean of W; stop when
            |s_new - s_old| <= 1e-3 h or after max_iter shifts; a seed
            whose W is empty is dropped; the mode is the last mean and its
            weight |W| of the last query;
  merge     modes ordered by weight (descending), ties by coordinates
            (lexicographically descending); walking that order, a mode
            still kept removes every later mode within distance h;
  K         the number of modes kept.

Distances are ((dx^2 + dy^2) + dz^2) (+ di^2 for a fourth coordinate) in
double, each operation rounded on its own.
"""
from __future__ import annotations

import numpy as np


def _sqdist(X, s):
    d = X - s
    q = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
    for j in range(2, X.shape[1]):
        q = q + d[:, j] * d[:, j]
    return q


def bin_seeds(X, h):
    """Seeds: the centres of the occupied bins of side h (lexicographic
    order of the bin indices)."""
    X = np.asarray(X, np.float64)
    b = np.unique(np.rint(X / h), axis=0)
    return b * h


def shift_seed(X, s, h, max_iter):
    """Mean shift of one seed: (mode, weight, iterations); weight 0 when the
    seed's first neighbourhood is empty (the seed is dropped)."""
    h2 = h * h
    stop = 1e-3 * h
    it = 0
    cnt = 0
    while True:
        inside = _sqdist(X, s) <= h2
        c = int(inside.sum())
        if c == 0:
            break
        cnt = c
        old = s
        s = X[inside].sum(axis=0) / c
        d = s - old
        dn = np.sqrt(float(_sqdist(d[None, :], np.zeros_like(d))[0]))
        if dn <= stop or it == max_iter:
            break
        it += 1
    return s, cnt, it


def merge(modes, weights, h):
    """Merge of converged modes given in seed order: the order is weight
    descending, then coordinates descending (lexicographic), then seed
    ascending (a stable sort); walking it, a mode still kept removes every
    later mode within distance h.  Returns (kept mask in seed order, the
    order as seed indices)."""
    modes = np.asarray(modes, np.float64)
    weights = np.asarray(weights)
    m = len(weights)
    order = sorted(range(m), key=lambda i: (weights[i], tuple(modes[i])), reverse=True)
    om = modes[order].reshape(m, -1)
    keep = np.ones(m, dtype=bool)
    h2 = float(h) * float(h)
    for i in range(m):
        if not keep[i]:
            continue
        near = _sqdist(om, om[i]) <= h2
        near[: i + 1] = False
        keep[near] = False
    mask = np.zeros(m, dtype=bool)
    mask[np.asarray(order, dtype=np.int64)[keep]] = True
    return mask, np.asarray(order, dtype=np.int64)


def gbms(X, bandwidth, max_iter=300):
    """Modes of the point cloud X (N x D, D = 3 or 4) for bandwidth h.
    Returns (modes (K, D) float64 in merge order, weights (K,) int64,
    all converged (mode, weight) pairs before the merge, in merge order)."""
    X = np.asarray(X, np.float64)
    h = float(bandwidth)
    res = []
    for s in bin_seeds(X, h):
        m, c, _ = shift_seed(X, s, h, max_iter)
        if c > 0:
            res.append((m, c))
    modes = np.array([r[0] for r in res]).reshape(-1, X.shape[1])
    w = np.array([r[1] for r in res], dtype=np.int64)
    mask, order = merge(modes, w, h)
    kept = order[mask[order]]
    return modes[kept], w[kept], (modes[order], w[order])
