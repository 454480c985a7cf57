"""Pins of the oracle's registration log-likelihood and its gradient.

* central finite differences of the oracle's own L (FP64);
* FP64 torch autograd of an independent expression (matrix exponential
  of the skew matrix for R, slogdet/solve Gaussian log-density,
  torch.logsumexp);
* EM fixed-point invariants: dL/dmu_b = 0 and dL/dpi_b = N;
* translation invariance: dL/dt = -sum_b dL/dmu_b;
* the K = 1 closed form dL/dmu = N Sigma^-1 (xbar - mu).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_00071_amd import synth


def _problem(seed=0, N=250, K=4):
    X, _, _ = synth.gaussian_blobs(seed, n_per=N // 2, k=2)
    X = X.astype(np.float64)
    w, mu, cov = synth.random_theta(K, seed + 1, spread=2.0, smin=0.8, smax=2.5)
    mu = mu + X.mean(axis=0)
    pose = synth.random_pose(seed + 2)
    return X, pose, w, mu, cov


def _fd(f, x, idx, h):
    xp = x.copy()
    xm = x.copy()
    xp[idx] += h
    xm[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


def test_gradient_vs_finite_differences():
    X, pose, w, mu, cov = _problem()
    g = oracle.loglik_grad(X, pose, w, mu, cov, grad_L=1.0)
    L = lambda **kw: oracle.loglik_pose(kw.get("X", X), kw.get("pose", pose),
                                        kw.get("w", w), kw.get("mu", mu),
                                        kw.get("cov", cov))
    for i in range(6):
        h = 1e-6
        fd = _fd(lambda p: L(pose=p), pose, i, h)
        assert abs(fd - g["pose"][i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g["pose"][i])
    for b in range(w.shape[0]):
        h = 1e-7 * w[b]
        fd = _fd(lambda v: L(w=v), w, b, h)
        assert abs(fd - g["w"][b]) <= 1e-6 * max(1.0, abs(fd))
        for i in range(3):
            fd = _fd(lambda v: L(mu=v), mu, (b, i), 1e-6)
            assert abs(fd - g["mu"][b, i]) <= 1e-6 * max(1.0, abs(fd))
        for i in range(3):
            for j in range(3):
                # f evaluated at sym(Sigma + h E_ij): perturb both (i,j), (j,i)
                def Lc(v, i=i, j=j):
                    return L(cov=0.5 * (v + np.transpose(v, (0, 2, 1))))
                fd = _fd(Lc, cov, (b, i, j), 1e-7)
                assert abs(fd - g["cov"][b, i, j]) <= 2e-6 * max(1.0, abs(fd))
    for n in (0, 17, 249):
        for i in range(3):
            fd = _fd(lambda v: L(X=v), X, (n, i), 1e-6)
            assert abs(fd - g["pts"][n, i]) <= 1e-6 * max(1.0, abs(fd))


def test_gradient_scales_with_upstream():
    X, pose, w, mu, cov = _problem(3)
    g1 = oracle.loglik_grad(X, pose, w, mu, cov, grad_L=1.0)
    g2 = oracle.loglik_grad(X, pose, w, mu, cov, grad_L=-2.5)
    for k in g1:
        np.testing.assert_allclose(g2[k], -2.5 * g1[k], rtol=1e-14)


def _torch_L(X, pose, w, mu, cov):
    om, t = pose[:3], pose[3:]
    zero = torch.zeros((), dtype=torch.float64)
    S = torch.stack([torch.stack([zero, -om[2], om[1]]),
                     torch.stack([om[2], zero, -om[0]]),
                     torch.stack([-om[1], om[0], zero])])
    R = torch.linalg.matrix_exp(S)
    Y = X @ R.T + t
    d = Y[:, None, :] - mu[None, :, :]                      # N,K,3
    sol = torch.linalg.solve(cov[None].expand(d.shape[0], -1, -1, -1),
                             d.unsqueeze(-1)).squeeze(-1)
    q = (d * sol).sum(-1)
    logdet = torch.linalg.slogdet(cov)[1]
    logp = torch.log(w)[None] - 0.5 * (3 * np.log(2 * np.pi) + logdet[None] + q)
    return torch.logsumexp(logp, dim=1).sum()


def test_gradient_vs_torch_autograd():
    X, pose, w, mu, cov = _problem(5, N=200, K=3)
    tX = torch.tensor(X, requires_grad=True)
    tp = torch.tensor(pose, requires_grad=True)
    tw = torch.tensor(w, requires_grad=True)
    tm = torch.tensor(mu, requires_grad=True)
    tc = torch.tensor(cov, requires_grad=True)
    Lt = _torch_L(tX, tp, tw, tm, tc)
    Lt.backward()
    Lo = oracle.loglik_pose(X, pose, w, mu, cov)
    assert abs(Lo - Lt.item()) <= 1e-12 * abs(Lo)
    g = oracle.loglik_grad(X, pose, w, mu, cov)
    np.testing.assert_allclose(g["pose"], tp.grad.numpy(), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(g["pts"], tX.grad.numpy(), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(g["w"], tw.grad.numpy(), rtol=1e-10)
    np.testing.assert_allclose(g["mu"], tm.grad.numpy(), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(g["cov"], tc.grad.numpy(), rtol=1e-9, atol=1e-9)


def test_small_angle_branch_continuity():
    X, _, w, mu, cov = _problem(6, N=100, K=3)
    for th in (5e-5, 2e-4):
        pose = np.array([th, -th / 2, th / 3, 0.1, 0.0, -0.1])
        g = oracle.loglik_grad(X, pose, w, mu, cov)
        L = lambda p: oracle.loglik_pose(X, p, w, mu, cov)
        for i in range(3):
            fd = _fd(L, pose, i, 1e-6)
            assert abs(fd - g["pose"][i]) <= 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("reg", [0.0, 1e-3])
def test_gradient_em_step_identities(reg):
    """At any theta, dL/dmu_b = Sigma_b^-1 sum_n gamma_nb (x_n - mu_b)
    = Sigma_b^-1 (N_b mu'_b - N0_b mu_b) and pi_b dL/dpi_b = N0_b, where
    mu', pi' come from the oracle's own (two-pass) M-step; so the gradient
    vanishes in mu and equals N in pi exactly at an EM fixed point."""
    X, _, _ = synth.gaussian_blobs(8, n_per=300, k=4)
    X = X.astype(np.float64)
    lab = synth.kmeanspp_labels(X, 4, 0)
    w, mu, cov, _ = oracle.fit(X, 4, reg, 3, labels=lab)
    g = oracle.loglik_grad(X, None, w, mu, cov)
    w1, mu1, _, _ = oracle.em_step(X, w, mu, cov, reg)
    N, K = X.shape[0], 4
    eps = 10 * np.finfo(np.float64).eps
    Nb = w1 * (N + K * eps)          # N0_b + eps
    N0 = Nb - eps
    np.testing.assert_allclose(g["w"] * w, N0, rtol=1e-10)
    for b in range(K):
        ref = np.linalg.solve(cov[b], Nb[b] * mu1[b] - N0[b] * mu[b])
        np.testing.assert_allclose(g["mu"][b], ref, rtol=1e-7,
                                   atol=1e-9 * np.abs(g["pts"]).sum())
    # translation invariance: dL/dt = sum_n dL/dy_n = -sum_b dL/dmu_b
    np.testing.assert_allclose(g["pose"][3:], g["pts"].sum(axis=0), rtol=1e-9, atol=1e-9)


def test_em_fixed_point_gradient_vanishes():
    X, _, _ = synth.gaussian_blobs(8, n_per=300, k=4)
    lab = synth.kmeanspp_labels(X, 4, 0)
    w, mu, cov, Lh = oracle.fit(X, 4, 1e-3, 3000, labels=lab)
    g = oracle.loglik_grad(X, None, w, mu, cov)
    assert np.abs(g["mu"]).max() <= 1e-6 * np.abs(g["pts"]).sum()
    np.testing.assert_allclose(g["w"], X.shape[0], rtol=1e-7)


def test_translation_invariance_off_fixed_point():
    X, pose, w, mu, cov = _problem(9)
    g = oracle.loglik_grad(X, pose, w, mu, cov)
    np.testing.assert_allclose(g["pose"][3:], -g["mu"].sum(axis=0), rtol=1e-10, atol=1e-8)


def test_k1_mean_gradient_closed_form():
    X, _, _ = synth.gaussian_blobs(10, n_per=200, k=1)
    X = X.astype(np.float64)
    mu = X.mean(axis=0) + np.array([[0.3, -0.2, 0.1]])
    cov = np.diag([0.5, 0.8, 1.1])[None]
    g = oracle.loglik_grad(X, None, np.array([1.0]), mu, cov)
    ref = X.shape[0] * np.linalg.solve(cov[0], X.mean(axis=0) - mu[0])
    np.testing.assert_allclose(g["mu"][0], ref, rtol=1e-11)
