"""GPU parity of the component-count estimate (gmm_meanshift, through the C
ABI) against the FP64 mean-shift oracle (oracle/gbms.py).

What is compared:
  * seeds: their number equals the oracle's occupied bins, in the same
    (lexicographic) order;
  * per seed: weight (the last neighbourhood's size) and iteration count
    identical, the mode within 1e-12 (max|x| + h) of the oracle's.  Both
    sides decide every neighbourhood, stop and merge in FP64 with the same
    operations; the sums that form a mean are added in different orders
    (numpy's against the GPU's fixed cell order), so the modes agree to a
    few units in the last place, and a decision could differ only for a
    point within that distance of a ball's surface;
  * the merge: the GPU's kept set equals the oracle's merge of the GPU's own
    seed modes (bit-exact: the same inputs), and K and the kept modes equal
    the oracle's end-to-end result (weights exact, modes as above);
  * at the full 320 x 240 depth-intensity frame (the paper's 2x-reduced
    image size) the per-seed check runs on a seeded sample of the seeds, and
    the merge by the two properties that make a kept set the greedy one
    (no two kept modes within h; every removed mode has a kept predecessor
    within h);
  * both forms of the shift (one wave per seed, four waves per seed) on one
    input with wide cells;
  * determinism (two calls bitwise equal), the error paths and the
    degenerate clouds (one point, identical points, points on bin edges,
    n = 0, max_iter = 0).
"""
import numpy as np
import pytest
import torch

from oracle import gbms as og
import paper_2307_00071_amd as gmm
from paper_2307_00071_amd import _lib, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _case(name):
    print("case:", name, flush=True)


def _run(X, h, max_iter=300):
    X32 = np.ascontiguousarray(X, np.float32)
    modes, w, info = gmm.meanshift(torch.from_numpy(X32).to(DEV), h, max_iter=max_iter,
                                   seeds=True)
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in info.items()}
    return modes.cpu().numpy(), w.cpu().numpy(), out


def _tol(X, h):
    return 1e-12 * (float(np.abs(X).max()) + h)


def _merge_order(modes, w):
    order = sorted(range(len(w)), key=lambda i: (w[i], tuple(modes[i])), reverse=True)
    return np.asarray(order, dtype=np.int64)


def _check_seeds(X, h, info, idx, max_iter=300):
    """Per-seed parity for the seed indices idx."""
    X64 = np.asarray(X, np.float32).astype(np.float64)
    seeds = og.bin_seeds(X64, h)
    assert info["n_seeds"] == seeds.shape[0]
    tol = _tol(X64, h)
    for i in idx:
        m, c, it = og.shift_seed(X64, seeds[i], h, max_iter)
        assert info["seed_weights"][i] == c, (i, info["seed_weights"][i], c)
        if c == 0:
            assert info["seed_status"][i] == 3
            continue
        assert info["seed_iters"][i] == it, (i, info["seed_iters"][i], it)
        err = np.abs(info["seed_modes"][i] - m).max()
        assert err <= tol, (i, err, tol)


def _check_merge_exact(h, info):
    """The GPU's kept set is the oracle's merge of the GPU's seed modes."""
    st = info["seed_status"]
    live = st != 3
    mask, _ = og.merge(info["seed_modes"][live], info["seed_weights"][live], h)
    np.testing.assert_array_equal(st[live] == 1, mask)


def _check_merge_properties(h, info):
    """Independence and predecessor domination (together: the greedy set)."""
    from scipy.spatial import cKDTree
    st = info["seed_status"]
    live = np.flatnonzero(st != 3)
    M = info["seed_modes"][live]
    W = info["seed_weights"][live].astype(np.int64)
    kept = st[live] == 1
    order = _merge_order(M, W)
    rank = np.empty(len(order), np.int64)
    rank[order] = np.arange(len(order))
    h2 = h * h
    tree = cKDTree(M[kept])
    kidx = np.flatnonzero(kept)
    for a, b in tree.query_pairs(h * (1 + 1e-9)):
        d = M[kidx[a]] - M[kidx[b]]
        assert og._sqdist(d[None, :], np.zeros_like(d))[0] > h2, "two kept modes within h"
    for i in np.flatnonzero(~kept):
        near = tree.query_ball_point(M[i], h * (1 + 1e-9))
        ok = False
        for a in near:
            j = kidx[a]
            d = M[i] - M[j]
            if og._sqdist(d[None, :], np.zeros_like(d))[0] <= h2 and rank[j] < rank[i]:
                ok = True
                break
        assert ok, "removed mode %d has no kept predecessor within h" % i


def _check_end_to_end(X, h, modes, w, max_iter=300):
    om, ow, _ = og.gbms(np.asarray(X, np.float32).astype(np.float64), h, max_iter)
    assert modes.shape == om.shape, (modes.shape, om.shape)
    order = _merge_order(modes, w)
    np.testing.assert_array_equal(w[order], ow)
    assert np.abs(modes[order] - om).max() <= _tol(X, h)


def _blobs(seed, k, n, d, sep, sigma):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-sep, sep, (k, d))
    X = np.concatenate([ci + sigma * rng.standard_normal((n, d)) for ci in c])
    return X.astype(np.float32)


@pytest.mark.parametrize("d,h,seed", [(3, 0.8, 0), (3, 0.35, 1), (4, 0.9, 2), (4, 0.5, 3)])
def test_blobs_match_oracle(d, h, seed):
    _case("blobs d=%d h=%g seed=%d" % (d, h, seed))
    X = _blobs(seed, k=6, n=150, d=d, sep=4.0, sigma=0.4)
    modes, w, info = _run(X, h)
    _check_seeds(X, h, info, range(info["n_seeds"]))
    _check_merge_exact(h, info)
    _check_end_to_end(X, h, modes, w)
    assert info["n_modes"] == modes.shape[0]


@pytest.mark.parametrize("d,n,h", [(4, 3000, 0.03), (3, 4000, 0.05), (4, 2500, 0.015)])
def test_depth_frame_subsample_matches_oracle(d, n, h):
    """Subsamples of the synthetic depth-intensity frame (many seeds, tiny
    neighbourhoods: the regime of the paper's bandwidths)."""
    _case("frame subsample d=%d n=%d h=%g" % (d, n, h))
    X = synth.depth_intensity_frame(0)[:, :d]
    rng = np.random.default_rng(5)
    X = np.ascontiguousarray(X[np.sort(rng.choice(X.shape[0], n, replace=False))])
    modes, w, info = _run(X, h)
    _check_seeds(X, h, info, range(info["n_seeds"]))
    _check_merge_exact(h, info)
    _check_end_to_end(X, h, modes, w)


def _frame_320x240():
    X = synth.depth_intensity_frame(0).reshape(480, 640, 4)[::2, ::2].reshape(-1, 4)
    return np.ascontiguousarray(X)


@pytest.mark.parametrize("h", [0.03, 0.015])
def test_full_frame_sampled(h):
    """The 320 x 240 frame (76,800 points, 4D): 150 sampled seeds against the
    oracle, the merge by its defining properties, and the exact oracle merge
    of the GPU's own seed modes at h = 0.03."""
    _case("full frame h=%g" % h)
    X = _frame_320x240()
    modes, w, info = _run(X, h)
    S = info["n_seeds"]
    rng = np.random.default_rng(11)
    idx = np.concatenate([[0, S - 1], rng.choice(S, 148, replace=False)])
    _check_seeds(X, h, info, idx)
    _check_merge_properties(h, info)
    if h == 0.03:
        _check_merge_exact(h, info)
    assert info["n_modes"] == int((info["seed_status"] == 1).sum()) == modes.shape[0]
    kept = np.flatnonzero(info["seed_status"] == 1)
    np.testing.assert_array_equal(modes, info["seed_modes"][kept])
    np.testing.assert_array_equal(w, info["seed_weights"][kept])
    print("seeds", S, "K", info["n_modes"], "rounds", info["rounds"],
          "max iters", info["max_iters"], flush=True)


def test_one_and_four_waves_per_seed(monkeypatch):
    """Both forms of the shift (one wave per seed; a block of four waves per
    seed, the default at most 16,384 seeds) on the 320 x 240 frame at h = 0.2:
    2,324 seeds whose neighbourhoods hold wide cells.  Each form against the
    oracle on sampled seeds (the slowest included), its merge exact, and the
    two forms' kept sets and weights equal, their modes within the per-seed
    bar of each other."""
    _case("one and four waves per seed h=0.2")
    X = _frame_320x240()
    h = 0.2
    out = {}
    for waves in ("1", "4"):
        monkeypatch.setenv("GMM_MS_SEED_WAVES", waves)
        modes, w, info = _run(X, h)
        S = info["n_seeds"]
        rng = np.random.default_rng(21)
        idx = np.unique(np.concatenate([[0, S - 1, int(np.argmax(info["seed_iters"]))],
                                        rng.choice(S, 16, replace=False)]))
        _check_seeds(X, h, info, idx)
        _check_merge_exact(h, info)
        out[waves] = (modes, w, info)
        print(waves, "wave(s): seeds", S, "K", info["n_modes"], "max iters",
              info["max_iters"], flush=True)
    (m1, w1, i1), (m4, w4, i4) = out["1"], out["4"]
    np.testing.assert_array_equal(i1["seed_status"], i4["seed_status"])
    np.testing.assert_array_equal(w1, w4)
    assert np.abs(m1 - m4).max() <= 2 * _tol(X, h)


def test_bitwise_deterministic():
    _case("determinism")
    X = _frame_320x240()[::3]
    a = _run(X, 0.02)
    b = _run(X, 0.02)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    for k in ("seed_modes", "seed_weights", "seed_iters", "seed_status"):
        np.testing.assert_array_equal(a[2][k], b[2][k])


def test_degenerate_clouds():
    _case("degenerate clouds")
    # one point: one seed, one mode at the point
    X = np.array([[0.25, -1.5, 3.0]], np.float32)
    modes, w, info = _run(X, 0.1)
    assert info["n_seeds"] == 1 and modes.shape == (1, 3) and w[0] == 1
    np.testing.assert_array_equal(modes[0], X[0].astype(np.float64))
    # identical points in three groups (the weight tie goes to the larger mode)
    X = np.array([[0.0, 0, 0]] * 5 + [[10.0, 0, 0]] * 3 + [[0.0, 20, 0]] * 5, np.float32)
    modes, w, info = _run(X, 1.0)
    _check_end_to_end(X, 1.0, modes, w)
    # coordinates on bin edges (x / h exactly k + 1/2: round half to even)
    h = 0.5
    X = (np.array([[0.25, 0.75, -0.25], [0.75, 1.25, -0.75], [1.25, -0.25, 0.25],
                   [-0.75, 0.25, 1.75]]) * 1.0).astype(np.float32)
    modes, w, info = _run(X, h)
    _check_seeds(X, h, info, range(info["n_seeds"]))
    _check_end_to_end(X, h, modes, w)
    # max_iter = 0: one mean per seed
    X = _blobs(7, k=3, n=60, d=4, sep=3.0, sigma=0.5)
    modes, w, info = _run(X, 0.7, max_iter=0)
    _check_seeds(X, 0.7, info, range(info["n_seeds"]), max_iter=0)
    assert info["max_iters"] == 0
    _check_end_to_end(X, 0.7, modes, w, max_iter=0)


def test_empty_and_errors():
    _case("empty and errors")
    modes, w, info = gmm.meanshift(torch.empty(0, 4, device=DEV), 0.1)
    assert modes.shape == (0, 4) and info["n_modes"] == 0 and info["n_seeds"] == 0
    X = torch.tensor([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]], device=DEV)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(_lib.GmmError) as e:
            gmm.meanshift(X, bad)
        assert e.value.status == _lib.GMM_ERR_INVALID_ARG
    with pytest.raises(_lib.GmmError) as e:
        gmm.meanshift(X, 0.1, max_iter=-1)
    assert e.value.status == _lib.GMM_ERR_INVALID_ARG
    # a bin index beyond the key range
    far = torch.tensor([[0.0, 0.0, 0.0], [5.0e4, 0.0, 0.0]], device=DEV)
    with pytest.raises(_lib.GmmError) as e:
        gmm.meanshift(far, 0.01)
    assert e.value.status == _lib.GMM_ERR_INVALID_ARG
    nanp = torch.tensor([[0.0, 0.0, 0.0], [float("nan"), 0.0, 0.0]], device=DEV)
    with pytest.raises(_lib.GmmError) as e:
        gmm.meanshift(nanp, 0.5)
    assert e.value.status == _lib.GMM_ERR_NONFINITE
    # the call still works after the errors
    modes, w, info = gmm.meanshift(X, 0.5)
    assert info["n_modes"] == 2
