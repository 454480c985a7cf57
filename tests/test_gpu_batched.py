"""GPU parity of gmm_fit_batched: every frame of a batched fit equals the
FP64 oracle's fit of that frame (same bar as single fits: one step 1e-5,
final log-likelihood 1e-4), and matches the per-frame gmm_fit."""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_00071_amd as gmm
from paper_2307_00071_amd import synth
from tests.parity import mixture_errors, rel as _rel

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _to(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to(DEV, dtype)


def _one_step_errors(r, X, ref):
    got = (r.weights.cpu().numpy(), r.means.cpu().numpy(), r.covariances.cpu().numpy())
    return mixture_errors(got, ref, X)


def _frames(count, seed, nmin, nmax, kmin, kmax):
    rng = np.random.default_rng(seed)
    out = []
    for f in range(count):
        X = synth.depth_frame(seed=seed + f)
        n = int(rng.integers(nmin, nmax + 1))
        k = int(rng.integers(kmin, kmax + 1))
        idx = np.sort(rng.choice(X.shape[0], n, replace=False))
        out.append((np.ascontiguousarray(X[idx]), k))
    return out


def test_batched_matches_oracle_per_frame():
    print("case: batched 6 frames", flush=True)
    frames = _frames(6, 500, 3000, 12000, 1, 150)
    frames.append((synth.gaussian_blobs(1, n_per=400)[0], 8))
    labs = [synth.kmeanspp_labels(X, k, 3) for X, k in frames]
    T = 12
    res = gmm.fit_batched([_to(X) for X, _ in frames], [k for _, k in frames],
                          iters=T, labels_list=[_to(l, torch.int32) for l in labs])
    torch.cuda.synchronize()
    for (X, k), lab, r in zip(frames, labs, res):
        w, mu, cov, Lr = oracle.fit(X, k, 1e-3, T, labels=lab)
        L = r.loglik.cpu().numpy()
        err = np.abs(L - Lr) / np.maximum(np.abs(Lr), X.shape[0])
        print(k, X.shape[0], err.max(), flush=True)
        assert err.max() <= 1e-4
        assert _rel(r.means.cpu().numpy(), mu) <= 1e-4


def test_batched_blocks_spanning_several_frames():
    """More tiles than resident blocks in one M-phase class, so blocks walk
    several frame segments; K in [65, 102] puts every frame in the class
    whose last point subset reads the zero pad column of the LDS rows."""
    print("case: batched multi-segment blocks", flush=True)
    rng = np.random.default_rng(42)
    frames = []
    for f in range(24):
        X = synth.depth_frame(seed=1200 + f)
        n = int(rng.integers(9000, 14000))
        idx = np.sort(rng.choice(X.shape[0], n, replace=False))
        frames.append((np.ascontiguousarray(X[idx]), int(rng.integers(65, 103))))
    labs = [synth.kmeanspp_labels(X, k, 3) for X, k in frames]
    T = 4
    res = gmm.fit_batched([_to(X) for X, _ in frames], [k for _, k in frames],
                          iters=T, labels_list=[_to(l, torch.int32) for l in labs])
    torch.cuda.synchronize()
    for (X, k), lab, r in zip(frames, labs, res):
        w, mu, cov, Lr = oracle.fit(X, k, 1e-3, T, labels=lab)
        L = r.loglik.cpu().numpy()
        err = np.abs(L - Lr) / np.maximum(np.abs(Lr), X.shape[0])
        assert err.max() <= 1e-4, (k, err.max())
        assert _rel(r.means.cpu().numpy(), mu) <= 1e-4


def test_batched_one_step_and_two_pass():
    print("case: batched one step", flush=True)
    frames = _frames(4, 700, 2000, 9000, 5, 120)
    thetas = []
    for X, k in frames:
        lab = synth.kmeanspp_labels(X, k, 4)
        w, mu, cov, _ = oracle.fit(X, k, 1e-3, 2, labels=lab)
        thetas.append(tuple(a.astype(np.float32) for a in (w, mu, cov)))
    for mode in ("shifted", "two_pass"):
        res = gmm.fit_batched([_to(X) for X, _ in frames], [k for _, k in frames],
                              iters=1, theta0_list=[tuple(_to(a) for a in t) for t in thetas],
                              moment_mode=mode)
        torch.cuda.synchronize()
        for (X, k), th, r in zip(frames, thetas, res):
            wr, mur, covr, L0 = oracle.em_step(X, *(a.astype(np.float64) for a in th), 1e-3)
            e = _one_step_errors(r, X, (wr, mur, covr))
            assert max(e.values()) <= 1e-5, (mode, k, e)
            assert abs(r.loglik[0].item() - L0) <= 1e-5 * max(abs(L0), X.shape[0])


def test_batched_equals_single_fits():
    """Same E-step/M-step per frame: batched and single fits agree to FP32
    summation-order rounding (different tile partitions)."""
    print("case: batched vs single", flush=True)
    frames = _frames(5, 900, 5000, 30000, 10, 200)
    labs = [synth.kmeanspp_labels(X, k, 5) for X, k in frames]
    T = 20
    res = gmm.fit_batched([_to(X) for X, _ in frames], [k for _, k in frames],
                          iters=T, labels_list=[_to(l, torch.int32) for l in labs])
    for (X, k), lab, r in zip(frames, labs, res):
        s = gmm.fit(_to(X), k, iters=T, labels=_to(lab, torch.int32))
        Lb, Ls = r.loglik.cpu().numpy(), s.loglik.cpu().numpy()
        assert np.abs(Lb - Ls).max() <= 1e-6 * np.abs(Ls).max()


def test_batched_deterministic_and_errors():
    print("case: batched determinism", flush=True)
    frames = _frames(3, 1100, 1000, 5000, 3, 60)
    labs = [synth.kmeanspp_labels(X, k, 6) for X, k in frames]
    args = ([_to(X) for X, _ in frames], [k for _, k in frames])
    a = gmm.fit_batched(*args, iters=5, labels_list=[_to(l, torch.int32) for l in labs])
    b = gmm.fit_batched(*args, iters=5, labels_list=[_to(l, torch.int32) for l in labs])
    for ra, rb in zip(a, b):
        for u, v in zip(ra, rb):
            np.testing.assert_array_equal(u.cpu().numpy(), v.cpu().numpy())
    from paper_2307_00071_amd import _lib
    bad = [l.copy() for l in labs]
    bad[1][7] = frames[1][1]        # label == K_f: out of range
    with pytest.raises(_lib.GmmError):
        gmm.fit_batched(*args, iters=2, labels_list=[_to(l, torch.int32) for l in bad])
    with pytest.raises(_lib.GmmError):
        gmm.fit_batched(*args[:1], [600, 3, 3], iters=1,
                        labels_list=[_to(l, torch.int32) for l in labs])


def test_batched_culled_matches_dense_batched(monkeypatch):
    """The culled batched passes (per-frame Morton order, tiles of 128
    points) against the dense batched kernel: same fit to FP32
    summation-order rounding, one step within the one-step bar."""
    print("case: batched culled vs dense", flush=True)
    frames = _frames(9, 1200, 2000, 40000, 8, 150)
    labs = [synth.kmeanspp_labels(X, k, 7) for X, k in frames]
    args = ([_to(X) for X, _ in frames], [k for _, k in frames])
    lab_t = [_to(l, torch.int32) for l in labs]
    monkeypatch.setenv("GMM_BATCH_CULL", "1")
    cull = gmm.fit_batched(*args, iters=10, labels_list=lab_t)
    monkeypatch.setenv("GMM_BATCH_CULL", "0")
    dense = gmm.fit_batched(*args, iters=10, labels_list=lab_t)
    for (X, k), rc, rd in zip(frames, cull, dense):
        Lc, Ld = rc.loglik.cpu().numpy(), rd.loglik.cpu().numpy()
        assert np.abs(Lc - Ld).max() <= 1e-6 * max(np.abs(Ld).max(), X.shape[0])
        assert _rel(rc.means.cpu().numpy(), rd.means.cpu().numpy().astype(np.float64)) <= 1e-5


def test_batched_culled_against_oracle(monkeypatch):
    """The culled batched passes meet the one-step bar per frame."""
    print("case: batched culled one step", flush=True)
    monkeypatch.setenv("GMM_BATCH_CULL", "1")
    frames = _frames(4, 1300, 3000, 25000, 10, 120)
    thetas = []
    for X, k in frames:
        lab = synth.kmeanspp_labels(X, k, 8)
        thetas.append(tuple(a.astype(np.float32) for a in oracle.fit(X, k, 1e-3, 2, labels=lab)[:3]))
    res = gmm.fit_batched([_to(X) for X, _ in frames], [k for _, k in frames], iters=1,
                          theta0_list=[tuple(_to(a) for a in th) for th in thetas])
    for (X, k), th, r in zip(frames, thetas, res):
        wr, mur, covr, L0 = oracle.em_step(X, *(a.astype(np.float64) for a in th), 1e-3)
        e = _one_step_errors(r, X, (wr, mur, covr))
        assert max(e.values()) <= 1e-5, (k, e)
        assert abs(r.loglik[0].item() - L0) <= 1e-5 * max(abs(L0), X.shape[0])


def test_batched_full_size_bench_workload():
    """The benchmark's batched workload itself (64 frames, N_f in [20k,
    300k], K_f in [16, 200], T = 20, one gmm_fit_batched call): every
    frame's final log-likelihood agrees with its own gmm_fit (any size),
    and three frames (the smallest, the largest N_f, the largest K_f) with
    the FP64 oracle."""
    print("case: batched bench workload 64 frames T=20", flush=True)
    frames = synth.batched_frames()
    T = 20
    labs = [synth.kmeanspp_labels(X, k, 1) for X, k in frames]
    pts = [_to(X) for X, _ in frames]
    ks = [k for _, k in frames]
    res = gmm.fit_batched(pts, ks, iters=T,
                          labels_list=[_to(l, torch.int32) for l in labs])
    torch.cuda.synchronize()
    for i, (p, k, l, r) in enumerate(zip(pts, ks, labs, res)):
        single = gmm.fit(p, k, iters=T, labels=_to(l, torch.int32))
        torch.cuda.synchronize()
        Lb = r.loglik.cpu().numpy()
        Ls = single.loglik.cpu().numpy()
        assert np.all(np.isfinite(Lb)), i
        assert abs(Lb[-1] - Ls[-1]) <= 1e-4 * max(abs(Ls[-1]), p.shape[0]), i
        assert abs(float(r.weights.sum()) - 1.0) <= 1e-5, i
    ns = [X.shape[0] for X, _ in frames]
    pick = sorted({int(np.argmin(ns)), int(np.argmax(ns)), int(np.argmax(ks))})
    for i in pick:
        X, k = frames[i]
        Lr = oracle.fit(X, k, 1e-3, T, labels=labs[i])[3]
        Lb = res[i].loglik.cpu().numpy()
        err = np.abs(Lb - Lr) / np.maximum(np.abs(Lr), X.shape[0])
        print("frame", i, X.shape[0], k, err.max(), flush=True)
        assert err.max() <= 1e-4


BATCH_SHAPES = ["bb512", "bb1024", "bc512p8s32", "bc512p8s64", "bc512p16s64"]


@pytest.mark.parametrize("shape", BATCH_SHAPES)
def test_every_batch_shape_one_step_parity(shape, monkeypatch):
    """Each soft-pass shape the batched autotuner may pick meets the
    one-step bar on every frame (per array and per component)."""
    from paper_2307_00071_amd import _lib
    monkeypatch.setenv("GMM_BATCH_SHAPE", shape)
    frames = _frames(5, 1400, 2000, 30000, 5, 220)
    ns, ks = [X.shape[0] for X, _ in frames], [k for _, k in frames]
    if _lib.batch_config(ns, ks) != shape:
        pytest.skip("shape %s cannot run these frames" % shape)
    print("case: batched shape %s" % shape, flush=True)
    thetas = []
    for X, k in frames:
        lab = synth.kmeanspp_labels(X, k, 9)
        thetas.append(tuple(a.astype(np.float32)
                            for a in oracle.fit(X, k, 1e-3, 2, labels=lab)[:3]))
    res = gmm.fit_batched([_to(X) for X, _ in frames], ks, iters=1,
                          theta0_list=[tuple(_to(a) for a in th) for th in thetas])
    torch.cuda.synchronize()
    for (X, k), th, r in zip(frames, thetas, res):
        wr, mur, covr, L0 = oracle.em_step(X, *(a.astype(np.float64) for a in th), 1e-3)
        e = _one_step_errors(r, X, (wr, mur, covr))
        assert max(e.values()) <= 1e-5, (shape, k, e)
        assert abs(r.loglik[0].item() - L0) <= 1e-5 * max(abs(L0), X.shape[0])


def test_batch_autotune_picks_caches_and_keeps_parity(monkeypatch, tmp_path):
    """With autotuning on, the first batched fit times every shape and keeps
    the fastest: the cache file names it, the library reports it, and the
    fit meets the final-L bar against the oracle; a second call reuses the
    tuned shape and agrees with a call forced to that shape bit for bit."""
    from paper_2307_00071_amd import _lib
    print("case: batched autotune", flush=True)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("GMM_AUTOTUNE_CACHE", str(cache))
    frames = _frames(6, 1500, 5000, 40000, 10, 150)
    ns, ks = [X.shape[0] for X, _ in frames], [k for _, k in frames]
    labs = [synth.kmeanspp_labels(X, k, 2) for X, k in frames]
    args = ([_to(X) for X, _ in frames], ks)
    lab_t = [_to(l, torch.int32) for l in labs]
    _lib.set_autotune(True)
    try:
        assert _lib.batch_config(ns, ks) == ""
        T = 8
        a = gmm.fit_batched(*args, iters=T, labels_list=lab_t)
        torch.cuda.synchronize()
        shape = _lib.batch_config(ns, ks)
        assert shape in BATCH_SHAPES, shape
        line = [l for l in cache.read_text().splitlines() if l.startswith("batch")][-1]
        assert line.split()[-1] == shape
        b = gmm.fit_batched(*args, iters=T, labels_list=lab_t)
        torch.cuda.synchronize()
    finally:
        _lib.set_autotune(False)
    monkeypatch.setenv("GMM_BATCH_SHAPE", shape)
    c = gmm.fit_batched(*args, iters=T, labels_list=lab_t)
    torch.cuda.synchronize()
    for ra, rb, rc in zip(a, b, c):
        for u, v, x in zip(ra, rb, rc):
            np.testing.assert_array_equal(u.cpu().numpy(), v.cpu().numpy())
            np.testing.assert_array_equal(u.cpu().numpy(), x.cpu().numpy())
    for (X, k), lab, r in zip(frames, labs, a):
        Lr = oracle.fit(X, k, 1e-3, T, labels=lab)[3]
        L = r.loglik.cpu().numpy()
        assert np.abs(L - Lr).max() <= 1e-4 * max(np.abs(Lr).max(), X.shape[0])
