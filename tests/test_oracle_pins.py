"""Pins of the FP64 oracle against things other than itself.

* brute force in 50-digit arithmetic on tiny inputs (eq. 1 ratio form,
  explicit determinant/adjugate density, weighted mean/scatter M-step);
* scipy's multivariate-normal log-density with scipy's logsumexp;
* scikit-learn's GaussianMixture, one EM iteration used as a black box;
* the K = 1 closed form (sample mean, biased sample covariance);
* invariants: responsibilities and weights sum to one, the covariance
  floor lambda, rigid-motion equivariance, permutation invariance;
* EM's monotone log-likelihood (exact M-step, lambda = 0).
"""
import warnings

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2307_00071_amd import synth
from tests import brute

EPS_N = 10 * np.finfo(np.float64).eps


def _tiny(seed, N=7, K=3):
    rng = np.random.default_rng(seed)
    w, mu, cov = synth.random_theta(K, seed, spread=1.0, smin=0.4, smax=1.2)
    X = rng.uniform(-1.5, 1.5, (N, 3))
    return X, w, mu, cov


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_estep_matches_bruteforce(seed):
    X, w, mu, cov = _tiny(seed)
    L, lse, lr = oracle.estep(X, w, mu, cov, want_logresp=True)
    Lb, G = brute.estep(X, w, mu, cov)
    assert abs(L - float(Lb)) <= 1e-13 * abs(float(Lb))
    for n in range(X.shape[0]):
        for b in range(w.shape[0]):
            ref = float(mp.log(G[n][b]))
            assert abs(lr[n, b] - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("seed", [3, 4])
def test_em_step_matches_bruteforce(seed):
    X, w, mu, cov = _tiny(seed, N=9, K=3)
    reg = 1e-3
    w1, mu1, cov1, L0 = oracle.em_step(X, w, mu, cov, reg)
    Lb, G = brute.estep(X, w, mu, cov)
    wb, mub, covb = brute.mstep(X, G, reg, mp.mpf(EPS_N))
    assert abs(L0 - float(Lb)) <= 1e-13 * abs(float(Lb))
    np.testing.assert_allclose(w1, np.array(wb, dtype=float), rtol=1e-12)
    np.testing.assert_allclose(mu1, np.array(mub, dtype=float), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(cov1, np.array(covb, dtype=float), rtol=1e-11, atol=1e-13)


def test_label_mstep_matches_bruteforce():
    X, _, _, _ = _tiny(5, N=10, K=3)
    lab = np.array([0, 1, 2, 0, 1, 2, 0, 0, 1, 2], dtype=np.int32)
    w, mu, cov = oracle.mstep_labels(X, lab, 3, 1e-3)
    G = [[mp.mpf(1) if lab[n] == b else mp.mpf(0) for b in range(3)]
         for n in range(10)]
    wb, mub, covb = brute.mstep(X, G, 1e-3, mp.mpf(EPS_N))
    np.testing.assert_allclose(w, np.array(wb, dtype=float), rtol=1e-13)
    np.testing.assert_allclose(mu, np.array(mub, dtype=float), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(cov, np.array(covb, dtype=float), rtol=1e-12, atol=1e-14)


def test_estep_matches_scipy():
    from scipy.special import logsumexp
    from scipy.stats import multivariate_normal
    rng = np.random.default_rng(11)
    K, N = 5, 300
    w, mu, cov = synth.random_theta(K, 12, spread=3.0)
    X = rng.uniform(-4, 4, (N, 3))
    logp = np.stack([np.log(w[b]) + multivariate_normal(mu[b], cov[b]).logpdf(X)
                     for b in range(K)], axis=1)
    ref_lse = logsumexp(logp, axis=1)
    L, lse, lr = oracle.estep(X, w, mu, cov, want_logresp=True)
    np.testing.assert_allclose(lse, ref_lse, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(lr, logp - ref_lse[:, None], rtol=1e-10, atol=1e-10)
    assert abs(L - ref_lse.sum()) <= 1e-12 * abs(L)


@pytest.mark.parametrize("K,seed", [(3, 0), (6, 1)])
def test_em_step_matches_sklearn(K, seed):
    from sklearn.mixture import GaussianMixture
    X, _, _ = synth.gaussian_blobs(seed, n_per=100)
    X = X.astype(np.float64)
    w0, mu0, cov0 = synth.random_theta(K, seed + 7, spread=1.0, smin=1.0, smax=3.0)
    mu0 = mu0 + X.mean(axis=0)
    reg = 1e-3
    gm = GaussianMixture(K, covariance_type="full", reg_covar=reg,
                         weights_init=w0, means_init=mu0,
                         precisions_init=np.linalg.inv(cov0), max_iter=1,
                         tol=0.0, n_init=1)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        gm.fit(X)
    w1, mu1, cov1, L0 = oracle.em_step(X, w0, mu0, cov0, reg)
    np.testing.assert_allclose(w1, gm.weights_, rtol=1e-12)
    np.testing.assert_allclose(mu1, gm.means_, rtol=1e-12)
    np.testing.assert_allclose(cov1, gm.covariances_, rtol=1e-11, atol=1e-14)
    # sklearn reports the mean per-point log-likelihood of the E-step
    assert abs(L0 / X.shape[0] - gm.lower_bound_) <= 1e-12 * abs(gm.lower_bound_)


def test_k1_closed_form_and_fixed_point():
    X, _, _ = synth.gaussian_blobs(2, n_per=200)
    X = X.astype(np.float64)
    N = X.shape[0]
    xbar = X.mean(axis=0)
    S = (X - xbar).T @ (X - xbar) / N
    for reg in (0.0, 1e-3):
        w, mu, cov, Lh = oracle.fit(X, 1, reg, 3, labels=np.zeros(N, np.int32))
        assert abs(w[0] - 1.0) < 1e-15
        np.testing.assert_allclose(mu[0], xbar, rtol=1e-13)
        np.testing.assert_allclose(cov[0], S + reg * np.eye(3), rtol=1e-12)
        # the K=1 update does not depend on theta: a fixed point after one step
        assert np.ptp(Lh) <= 1e-12 * abs(Lh[0])
    # lambda = 0: L = -N/2 (3 ln 2pi + ln|S| + 3)
    Lcf = -N / 2 * (3 * np.log(2 * np.pi) + np.log(np.linalg.det(S)) + 3)
    w, mu, cov, Lh0 = oracle.fit(X, 1, 0.0, 1, labels=np.zeros(N, np.int32))
    assert abs(Lh0[-1] - Lcf) <= 1e-11 * abs(Lcf)


def test_invariants():
    X, _, _ = synth.gaussian_blobs(3, n_per=150)
    X = X.astype(np.float64)
    K, reg = 5, 2e-3
    w0, mu0, cov0 = synth.random_theta(K, 4, spread=4.0, smin=0.5, smax=2.0)
    mu0 += 5.0
    L, lse, lr = oracle.estep(X, w0, mu0, cov0, want_logresp=True)
    np.testing.assert_allclose(np.exp(lr).sum(axis=1), 1.0, rtol=1e-13)
    w1, mu1, cov1, _ = oracle.em_step(X, w0, mu0, cov0, reg)
    assert abs(w1.sum() - 1.0) < 1e-14
    for b in range(K):
        assert np.linalg.eigvalsh(cov1[b]).min() >= reg * (1 - 1e-12)
        np.testing.assert_allclose(cov1[b], cov1[b].T, rtol=0, atol=0)
        # a weighted mean lies inside the bounding box of the points
        assert np.all(mu1[b] >= X.min(axis=0) - 1e-9)
        assert np.all(mu1[b] <= X.max(axis=0) + 1e-9)
    # N_b: sum of weights * total count
    Nb = np.exp(lr).sum(axis=0)
    np.testing.assert_allclose(w1 * (X.shape[0] + K * EPS_N), Nb + EPS_N, rtol=1e-12)


def test_rigid_motion_equivariance():
    X, _, _ = synth.gaussian_blobs(4, n_per=120)
    X = X.astype(np.float64)
    K, reg = 4, 1e-3
    w0, mu0, cov0 = synth.random_theta(K, 5, spread=3.0, smin=0.5, smax=2.0)
    mu0 += 5.0
    R = synth.haar_rotation(np.random.default_rng(9))
    t = np.array([1.5, -2.0, 0.75])
    Xt = X @ R.T + t
    mu0t = mu0 @ R.T + t
    cov0t = R @ cov0 @ R.T
    w1, mu1, cov1, L0 = oracle.em_step(X, w0, mu0, cov0, reg)
    w2, mu2, cov2, L0t = oracle.em_step(Xt, w0, mu0t, cov0t, reg)
    assert abs(L0 - L0t) <= 1e-10 * abs(L0)
    np.testing.assert_allclose(w2, w1, rtol=1e-9)
    np.testing.assert_allclose(mu2, mu1 @ R.T + t, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(cov2, R @ cov1 @ R.T, rtol=1e-8, atol=1e-11)


def test_permutation_invariance():
    X, _, _ = synth.gaussian_blobs(5, n_per=100)
    X = X.astype(np.float64)
    K, reg = 4, 1e-3
    w0, mu0, cov0 = synth.random_theta(K, 6, spread=3.0, smin=0.5, smax=2.0)
    mu0 += 5.0
    rng = np.random.default_rng(1)
    pn = rng.permutation(X.shape[0])
    pk = rng.permutation(K)
    w1, mu1, cov1, L0 = oracle.em_step(X, w0, mu0, cov0, reg)
    w2, mu2, cov2, L2 = oracle.em_step(X[pn], w0[pk], mu0[pk], cov0[pk], reg)
    assert abs(L0 - L2) <= 1e-12 * abs(L0)
    np.testing.assert_allclose(w2, w1[pk], rtol=1e-12)
    np.testing.assert_allclose(mu2, mu1[pk], rtol=1e-12)
    np.testing.assert_allclose(cov2, cov1[pk], rtol=1e-10, atol=1e-14)


def test_monotone_loglik_exact_mstep():
    X, _, _ = synth.gaussian_blobs(6)
    lab = synth.kmeanspp_labels(X, 8, 1)
    _, _, _, Lh = oracle.fit(X, 8, 0.0, 30, labels=lab)
    d = np.diff(Lh)
    assert np.all(d >= -1e-12 * abs(Lh[-1])), d.min()
    # a looser start (fewer, overlapping components) still climbs
    lab3 = synth.kmeanspp_labels(X, 3, 2)
    _, _, _, Lh3 = oracle.fit(X, 3, 0.0, 30, labels=lab3)
    assert np.all(np.diff(Lh3) >= -1e-12 * abs(Lh3[-1]))
    assert Lh3[-1] > Lh3[0]


def test_fit_from_theta_equals_fit_from_labels():
    X, _, _ = synth.gaussian_blobs(7, n_per=200)
    lab = synth.kmeanspp_labels(X, 8, 3)
    w0, mu0, cov0 = oracle.mstep_labels(X, lab, 8, 1e-3)
    a = oracle.fit(X, 8, 1e-3, 5, labels=lab)
    b = oracle.fit(X, 8, 1e-3, 5, theta0=(w0, mu0, cov0))
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def test_error_statuses():
    X = np.zeros((4, 3))
    w = np.array([1.0])
    mu = np.zeros((1, 3))
    bad = -np.eye(3)[None]
    with pytest.raises(oracle.OracleError, match="SPD"):
        oracle.estep(X, w, mu, bad)
    with pytest.raises(oracle.OracleError, match="invalid"):
        oracle.estep(X, np.array([0.0]), mu, np.eye(3)[None])
    with pytest.raises(oracle.OracleError, match="invalid"):
        oracle.mstep_labels(X, np.array([0, 1, 0, 0]), 1, 1e-3)
