"""GPU parity of gmm_loglik / gmm_loglik_backward (registration of a moved
point cloud against a fixed GMM) against the FP64 oracle.

Every gradient entry is compared on its own, against the scale of the terms
that make it up (where terms cancel, a relative bar on the result would
measure the cancellation, not the arithmetic):
  * g_w[b] = N_b / pi_b (a plain sum of responsibilities): relative 1e-5;
  * g_mu[b] = Sigma_b^-1 sum_n g_nb d_nb: each term has size about
    |Sigma_b^-1/2| per point, so the scale is N_b |Sigma_b^-1|_2^(1/2);
  * g_cov[b] = 1/2 Sigma^-1 (sum g d d^T) Sigma^-1 - 1/2 N_b Sigma^-1: two
    terms of size N_b |Sigma_b^-1|_2 that nearly cancel near a fit;
  * g_pts[n] = -sum_b g_nb Sigma_b^-1 d_nb: scale |g_pts[n]| plus the RMS
    over points (a point between two components feels cancelling pulls);
  * g_pose: the rotation and translation parts each on the scale of their
    largest entry;
with N_b = g_w[b] w_b.  The bar is |gpu - oracle| <= 1e-5 scale + 1e-4 |oracle|
for the component sums and the pose (FP64 sums of FP32 terms whose relative
rounding is a few 1e-7), plus a floor of 1e-7 of the array's largest scale
(1e-6 for g_w): a component holding a vanishing share of the points is
built from far-tail responsibilities, whose FP32 exponentials lose relative
precision and flush to zero below 2^-126 while the oracle keeps them; and
1e-4 (scale + |oracle|) for the per-point
gradients (one FP32 evaluation each: the transformed point y = R x + t is
rounded to FP32, an absolute error near 1e-6 m that is ~3e-5 of a 3 cm
standard deviation).  L must agree to 1e-5 relative (floor N).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_00071_amd as gmm
from paper_2307_00071_amd import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _to(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to(DEV, dtype)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) /
                 max(np.linalg.norm(b), 1e-300))


def _case(name):
    print("case:", name, flush=True)


def _registration_problem(n_src, K, seed=0, fit_n=30000, fit_iters=5):
    """Target GMM fitted (oracle, FP64) on one render of a scene; source =
    n_src points of a second noisy render of the same scene; random pose."""
    X = synth.depth_frame(seed)
    rng = np.random.default_rng(seed + 101)
    sub = np.ascontiguousarray(X[np.sort(rng.choice(X.shape[0], fit_n, replace=False))])
    lab = synth.kmeanspp_labels(sub, K, seed + 1)
    w, mu, cov, _ = oracle.fit(sub, K, 1e-3, fit_iters, labels=lab)
    th = (w.astype(np.float32), mu.astype(np.float32), cov.astype(np.float32))
    Y = synth.depth_frame(seed, noise_seed=seed + 7)
    src = np.ascontiguousarray(Y[np.sort(rng.choice(Y.shape[0], n_src, replace=False))])
    pose = synth.random_pose(seed + 2).astype(np.float32)
    return src, pose, th


def _scales(gr, th64):
    """Per-entry scales of the oracle gradient (see the module notes)."""
    w, mu, cov = th64
    K = w.shape[0]
    Nb = gr["w"] * w
    lam = np.linalg.eigvalsh(np.linalg.inv(cov)).max(axis=1)   # |Sigma^-1|_2
    gp = gr["pts"]
    pnorm = np.linalg.norm(gp, axis=1)
    rms = float(np.sqrt((pnorm ** 2).mean()))
    sc = {"w": np.abs(gr["w"]),
          "mu": np.repeat((Nb * np.sqrt(lam))[:, None], 3, axis=1),
          "cov": np.broadcast_to((Nb * lam)[:, None, None], (K, 3, 3)),
          "pts": np.repeat((pnorm + rms)[:, None], 3, axis=1)}
    if "pose" in gr:
        p = np.abs(gr["pose"])
        sc["pose"] = np.concatenate([np.full(3, p[:3].max()), np.full(3, p[3:].max())])
    return sc


def _elementwise(g, gr, th64, keys):
    """max over entries of |gpu - oracle| / bar, bar per the module notes."""
    sc = _scales(gr, th64)
    out = {}
    for key in keys:
        a = np.asarray(g[key], np.float64)
        r = gr[key]
        if key == "w":
            bar = 1e-5 * sc["w"] + 1e-6 * sc["w"].max() + 1e-30
        elif key == "pts":
            bar = 1e-4 * (sc["pts"] + np.abs(r)) + 1e-30
        else:
            bar = 1e-5 * sc[key] + 1e-4 * np.abs(r) + 1e-7 * sc[key].max() + 1e-30
        out[key] = float((np.abs(a - r) / bar).max())
    return out


def _check(src, pose, th):
    th64 = tuple(a.astype(np.float64) for a in th)
    p64 = None if pose is None else pose.astype(np.float64)
    Lr = oracle.loglik_pose(src, p64, *th64)
    gr = oracle.loglik_grad(src, p64, *th64, grad_L=1.0)
    tpose = None if pose is None else _to(pose)
    L = gmm.loglik(_to(src), *(_to(a) for a in th), pose6=tpose)
    g = gmm.loglik_backward(_to(src), *(_to(a) for a in th), pose6=tpose)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if v is not None}
    N = src.shape[0]
    keys = ("pts", "w", "mu", "cov") + (("pose",) if pose is not None else ())
    errs = {"L": abs(L.item() - Lr) / max(abs(Lr), N)}
    fro = {k: _rel(g[k], gr[k]) for k in keys}
    ew = _elementwise(g, gr, th64, keys)
    print("L", errs["L"], "frobenius", fro, "element-wise / bar", ew, flush=True)
    assert errs["L"] <= 1e-5, errs
    for key, e in ew.items():
        assert e <= 1.0, (key, e, ew)
    return g, gr


def test_registration_full_size_forward_backward():
    """The registration workload: K = 200 target, N = 100,000 source points,
    |omega| <= 0.3 rad, |t| <= 0.5 m."""
    _case("registration N=100000 K=200")
    src, pose, th = _registration_problem(100000, 200)
    _check(src, pose, th)


@pytest.mark.parametrize("n,K", [(5000, 1), (777, 16), (20011, 64), (3000, 300)])
def test_registration_sizes(n, K):
    _case("registration n=%d K=%d" % (n, K))
    src, pose, th = _registration_problem(n, K, seed=K, fit_n=max(4000, 4 * K))
    _check(src, pose, th)


def test_identity_pose_and_small_angle():
    _case("identity / small angle")
    src, _, th = _registration_problem(8000, 32, seed=3, fit_n=8000)
    _check(src, None, th)
    _check(src, np.array([3e-5, -2e-5, 1e-5, 0.05, 0.0, -0.02], np.float32), th)


def test_autograd_function_matches_backward():
    _case("autograd")
    src, pose, th = _registration_problem(20000, 50, seed=5, fit_n=10000)
    pts = _to(src).requires_grad_(True)
    tp = _to(pose).requires_grad_(True)
    tw, tm, tc = (_to(a).requires_grad_(True) for a in th)
    L = gmm.GMMLogLik.apply(pts, tp, tw, tm, tc)
    (2.5 * L).backward()
    g = gmm.loglik_backward(_to(src), *(_to(a) for a in th), pose6=_to(pose))
    for key, t in (("pts", pts), ("pose", tp), ("w", tw), ("mu", tm), ("cov", tc)):
        np.testing.assert_allclose(t.grad.cpu().numpy(), 2.5 * g[key].cpu().numpy(),
                                   rtol=1e-6, atol=1e-6 * float(g[key].abs().max()))


def test_pose_gradient_vs_gpu_finite_differences():
    """Central differences of the GPU's own L (FP64 sums of FP32 terms),
    Richardson-extrapolated over steps 2h and h (truncation O(h^4)): an
    independent check of the pose gradient's sign and scale.  Rounding of
    the FP32 E-step puts noise of order 1e-8 |L| on each L, which is
    ~1e-3 of the smallest pose-gradient entry at these steps."""
    _case("gpu fd")
    src, pose, th = _registration_problem(30000, 40, seed=6, fit_n=10000)
    g = gmm.loglik_backward(_to(src), *(_to(a) for a in th), pose6=_to(pose))
    gp = g["pose"].cpu().numpy()
    args = (_to(src), *(_to(a) for a in th))

    def central(i, h):
        pp, pm = pose.astype(np.float64), pose.astype(np.float64)
        pp[i] += h
        pm[i] -= h
        Lp = gmm.loglik(*args, pose6=_to(pp)).item()
        Lm = gmm.loglik(*args, pose6=_to(pm)).item()
        # the steps as float32 actually applied
        hh = 0.5 * (float(np.float32(pp[i])) - float(np.float32(pm[i])))
        return (Lp - Lm) / (2 * hh)

    for i in range(6):
        h = 2e-3
        fd = (4.0 * central(i, h / 2) - central(i, h)) / 3.0
        print(i, fd, gp[i], flush=True)
        assert abs(fd - gp[i]) <= 5e-3 * max(abs(fd), np.abs(gp).max() * 1e-2), (i, fd, gp[i])


def test_grad_scaling_by_upstream():
    _case("upstream scaling")
    src, pose, th = _registration_problem(5000, 20, seed=8, fit_n=5000)
    args = (_to(src), *(_to(a) for a in th))
    g1 = gmm.loglik_backward(*args, pose6=_to(pose))
    g2 = gmm.loglik_backward(*args, pose6=_to(pose),
                             grad_L=torch.tensor(-3.0, dtype=torch.float64, device=DEV))
    for key in g1:
        np.testing.assert_allclose(g2[key].cpu().numpy(), -3.0 * g1[key].cpu().numpy(),
                                   rtol=1e-6, atol=1e-30)


@pytest.mark.parametrize("shape", ["b1024t128", "b512t128"])
def test_backward_under_forced_128_point_forward_shape(shape, monkeypatch):
    """The backward kernel tiles by 64 points whatever forward shape is
    forced or tuned: every point must reach the gradients."""
    _case("backward with GMM_TILE_SHAPE=%s" % shape)
    monkeypatch.setenv("GMM_TILE_SHAPE", shape)
    src, pose, th = _registration_problem(20011, 64, seed=11, fit_n=8000)
    _check(src, pose, th)


def test_device_errors_are_raised_forward_and_backward():
    """A covariance that is not SPD, a weight <= 0 and a non-finite point are
    device-side conditions: loglik / loglik_backward raise GmmError with the
    status, and a failed component's gradients are NaN (not stale memory)."""
    from paper_2307_00071_amd._lib import GmmError
    _case("device errors")
    src, pose, th = _registration_problem(4000, 8, seed=12, fit_n=4000)
    w, mu, cov = (a.copy() for a in th)
    bad = cov.copy()
    bad[3] = np.diag([1.0, -1.0, 1.0]).astype(np.float32)   # indefinite
    for fn in (lambda c: gmm.loglik(_to(src), _to(w), _to(mu), _to(c), pose6=_to(pose)),
               lambda c: gmm.loglik_backward(_to(src), _to(w), _to(mu), _to(c),
                                             pose6=_to(pose))):
        with pytest.raises(GmmError) as ei:
            fn(bad)
        assert ei.value.status == 2, ei.value          # GMM_ERR_NOT_SPD
    g = gmm.loglik_backward(_to(src), _to(w), _to(mu), _to(bad), pose6=_to(pose),
                            check=False)
    torch.cuda.synchronize()
    for key, shp in (("w", ()), ("mu", (3,)), ("cov", (3, 3))):
        v = g[key].cpu().numpy()
        assert np.isnan(v[3]).all(), key
        assert np.isfinite(np.delete(v, 3, axis=0)).all(), key
    wneg = w.copy()
    wneg[1] = 0.0
    with pytest.raises(GmmError) as ei:
        gmm.loglik(_to(src), _to(wneg), _to(mu), _to(cov))
    assert ei.value.status == 1, ei.value              # GMM_ERR_INVALID_ARG
    nanpts = src.copy()
    nanpts[17, 1] = np.nan
    for fn in (lambda: gmm.loglik(_to(nanpts), _to(w), _to(mu), _to(cov)),
               lambda: gmm.loglik_backward(_to(nanpts), _to(w), _to(mu), _to(cov))):
        with pytest.raises(GmmError) as ei:
            fn()
        assert ei.value.status == 3, ei.value          # GMM_ERR_NONFINITE
    # a good call on the same process afterwards is unaffected
    _check(src, pose, th)
