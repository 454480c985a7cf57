"""Pins of the 4D oracle (oracle/gmm4.py: EM of the (x, y, z, intensity)
mixture, conditional intensity, joint sampling) against things other than
itself:

* 50-digit brute force on tiny inputs (mpmath: density from the explicit
  determinant and inverse, responsibilities as the ratio of eq. 1,
  weighted mean / scatter M-step);
* scipy's multivariate-normal log-density and logsumexp;
* scikit-learn's GaussianMixture, one EM iteration as a black box, in 4D;
* the K = 1 closed form and its fixed point; monotone L (lambda = 0);
* the 3D C oracle: the D-generic code on 3D data agrees with it;
* conditional intensity: 30-digit quadrature of the joint density over the
  intensity axis (E = int i p(x, i) di / int p(x, i) di, V likewise), and
  the cases that reduce to a plain formula (no cross-covariance);
* joint sampling: component picks against an exact rational running sum,
  one component with identity covariance (sample = mu + z), and sample
  moments of many draws against the mixture's mean and covariance.
"""
import warnings
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import gmm4
from paper_2307_00071_amd import synth

mp.mp.dps = 50
EPS_N = 10 * np.finfo(np.float64).eps


def _theta4(K, seed, spread=1.0, smin=0.3, smax=1.1):
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.2, 1.0, K)
    w /= w.sum()
    mu = rng.uniform(-spread, spread, (K, 4))
    cov = np.empty((K, 4, 4))
    for b in range(K):
        Q, R = np.linalg.qr(rng.standard_normal((4, 4)))
        Q = Q * np.sign(np.diag(R))
        s = rng.uniform(smin, smax, 4)
        cov[b] = Q @ np.diag(s * s) @ Q.T
        cov[b] = 0.5 * (cov[b] + cov[b].T)
    return w, mu, cov


def _mp_density(x, mu, S):
    S = mp.matrix([[mp.mpf(float(v)) for v in row] for row in S])
    d = mp.matrix([mp.mpf(float(x[i])) - mp.mpf(float(mu[i])) for i in range(len(x))])
    q = (d.T * mp.inverse(S) * d)[0]
    return mp.exp(-q / 2) / mp.sqrt((2 * mp.pi) ** len(x) * mp.det(S))


def _mp_estep(X, w, mu, cov):
    L = mp.mpf(0)
    G = []
    for x in X:
        t = [mp.mpf(float(w[b])) * _mp_density(x, mu[b], cov[b]) for b in range(len(w))]
        tot = sum(t)
        L += mp.log(tot)
        G.append([v / tot for v in t])
    return L, G


@pytest.mark.parametrize("seed", [0, 1])
def test_estep_and_mstep_match_bruteforce(seed):
    w, mu, cov = _theta4(3, seed)
    X = np.random.default_rng(seed + 10).uniform(-1.5, 1.5, (8, 4))
    L, lse, g = gmm4.estep(X, w, mu, cov)
    Lb, G = _mp_estep(X, w, mu, cov)
    assert abs(L - float(Lb)) <= 1e-13 * abs(float(Lb))
    np.testing.assert_allclose(g, np.array(G, dtype=float), rtol=1e-12, atol=1e-15)
    reg = 1e-3
    w1, mu1, cov1 = gmm4.mstep(X, g, reg)
    Gm = [[mp.mpf(v) for v in row] for row in G]
    Xm = [[mp.mpf(float(v)) for v in row] for row in X]
    Nb = [sum(Gm[n][b] for n in range(8)) + mp.mpf(EPS_N) for b in range(3)]
    for b in range(3):
        mb = [sum(Gm[n][b] * Xm[n][i] for n in range(8)) / Nb[b] for i in range(4)]
        np.testing.assert_allclose(mu1[b], np.array(mb, dtype=float), rtol=1e-11, atol=1e-13)
        for i in range(4):
            for j in range(4):
                v = sum(Gm[n][b] * (Xm[n][i] - mb[i]) * (Xm[n][j] - mb[j])
                        for n in range(8)) / Nb[b] + (reg if i == j else 0)
                assert abs(cov1[b, i, j] - float(v)) <= 1e-11 * max(1e-2, abs(float(v)))
        assert abs(w1[b] - float(Nb[b] / sum(Nb))) <= 1e-13


def test_estep_matches_scipy():
    from scipy.special import logsumexp
    from scipy.stats import multivariate_normal
    w, mu, cov = _theta4(5, 3, spread=2.0)
    X = np.random.default_rng(4).normal(0, 2, (300, 4))
    L, lse, _ = gmm4.estep(X, w, mu, cov)
    ref = np.stack([np.log(w[b]) + multivariate_normal(mu[b], cov[b]).logpdf(X)
                    for b in range(5)], axis=1)
    np.testing.assert_allclose(lse, logsumexp(ref, axis=1), rtol=1e-12)
    assert abs(L - logsumexp(ref, axis=1).sum()) <= 1e-11 * abs(L)


def test_one_iteration_matches_sklearn_4d():
    from sklearn.mixture import GaussianMixture
    X = synth.depth_intensity_frame(2).astype(np.float64)
    X = X[np.random.default_rng(5).choice(X.shape[0], 3000, replace=False)]
    K, reg = 6, 1e-3
    lab = np.random.default_rng(6).integers(0, K, X.shape[0])
    w, mu, cov = gmm4.mstep_labels(X, lab, K, reg)
    w1, mu1, cov1, _ = gmm4.em_step(X, w, mu, cov, reg)
    gm = GaussianMixture(K, covariance_type="full", reg_covar=reg, max_iter=1,
                         tol=0.0, weights_init=w, means_init=mu,
                         precisions_init=np.linalg.inv(cov))
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        gm.fit(X)
    np.testing.assert_allclose(w1, gm.weights_, rtol=1e-12)
    np.testing.assert_allclose(mu1, gm.means_, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(cov1, gm.covariances_, rtol=1e-10, atol=1e-13)


def test_k1_closed_form_and_fixed_point():
    X = synth.depth_intensity_frame(1)[::37].astype(np.float64)
    reg = 2e-3
    w, mu, cov, L = gmm4.fit(X, 1, reg, 3, labels=np.zeros(X.shape[0], np.int64))
    xb = X.mean(axis=0)
    S = (X - xb).T @ (X - xb) / X.shape[0] + reg * np.eye(4)
    np.testing.assert_allclose(mu[0], xb, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(cov[0], S, rtol=1e-10, atol=1e-13)
    assert abs(w[0] - 1.0) <= 1e-15
    assert np.ptp(L) <= 1e-9 * abs(L[0])


def test_monotone_loglik_without_regulariser():
    X = synth.depth_intensity_frame(3)[::53].astype(np.float64)
    lab = np.random.default_rng(1).integers(0, 7, X.shape[0])
    _, _, _, L = gmm4.fit(X, 7, 0.0, 15, labels=lab)
    assert np.all(np.diff(L) >= -1e-10 * abs(L[-1]))


def test_generic_code_on_3d_data_agrees_with_the_c_oracle():
    X = synth.depth_frame(4)[::61].astype(np.float64)
    lab = synth.kmeanspp_labels(X, 9, 2)
    a = gmm4.fit(X, 9, 1e-3, 4, labels=lab)
    b = oracle.fit(X, 9, 1e-3, 4, labels=lab)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, rtol=1e-10, atol=1e-13)


# ------------------------------------------------------ conditional intensity

def _quad_conditional(x, w, mu, cov):
    """E and V of the intensity at x by 30-digit quadrature of the joint
    density along the intensity axis (inverse and determinant of each
    covariance formed once, by mpmath's LU)."""
    with mp.workdps(30):
        comps = []
        for b in range(len(w)):
            S = mp.matrix([[mp.mpf(float(v)) for v in row] for row in cov[b]])
            comps.append((mp.mpf(float(w[b])), [mp.mpf(float(v)) for v in mu[b]],
                          mp.inverse(S), 1 / mp.sqrt((2 * mp.pi) ** 4 * mp.det(S))))
        xm = [mp.mpf(float(v)) for v in x]

        def p(i):
            tot = mp.mpf(0)
            for wb, mb, Si, nc in comps:
                d = [xm[0] - mb[0], xm[1] - mb[1], xm[2] - mb[2], i - mb[3]]
                q = sum(d[r] * Si[r, c] * d[c] for r in range(4) for c in range(4))
                tot += wb * nc * mp.exp(-q / 2)
            return tot

        lo, hi = -12, 12
        Z = mp.quad(p, [lo, 0, hi])
        E = mp.quad(lambda i: i * p(i), [lo, 0, hi]) / Z
        V = mp.quad(lambda i: (i - E) ** 2 * p(i), [lo, 0, hi]) / Z
        return float(E), float(V)


@pytest.mark.parametrize("seed", [0, 1])
def test_conditional_matches_quadrature(seed):
    w, mu, cov = _theta4(3, seed + 20, spread=1.0, smin=0.4, smax=1.0)
    locs = np.random.default_rng(seed).uniform(-1, 1, (3, 3))
    E, V, beta = gmm4.color_conditional(locs, w, mu, cov)
    np.testing.assert_allclose(beta.sum(axis=1), 1.0, rtol=1e-14)
    for m in range(3):
        Eq, Vq = _quad_conditional(locs[m], w, mu, cov)
        assert abs(E[m] - Eq) <= 1e-10 * max(1.0, abs(Eq)), (m, E[m], Eq)
        assert abs(V[m] - Vq) <= 1e-9 * Vq, (m, V[m], Vq)


def test_conditional_without_cross_covariance():
    """Sigma_b^xi = 0: each component's conditional mean is mu_b^i and its
    variance Sigma_b^ii, mixed with the 3D marginal responsibilities; with
    one component E = mu^i and V = Sigma^ii everywhere."""
    from scipy.stats import multivariate_normal
    w, mu, cov = _theta4(4, 7)
    cov[:, :3, 3] = 0.0
    cov[:, 3, :3] = 0.0
    locs = np.random.default_rng(8).uniform(-1, 1, (50, 3))
    E, V, beta = gmm4.color_conditional(locs, w, mu, cov)
    r = np.stack([w[b] * multivariate_normal(mu[b, :3], cov[b, :3, :3]).pdf(locs)
                  for b in range(4)], axis=1)
    r /= r.sum(axis=1, keepdims=True)
    np.testing.assert_allclose(beta, r, rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(E, r @ mu[:, 3], rtol=1e-12)
    np.testing.assert_allclose(V, r @ (cov[:, 3, 3] + mu[:, 3] ** 2) - (r @ mu[:, 3]) ** 2,
                               rtol=1e-10, atol=1e-14)
    E1, V1, _ = gmm4.color_conditional(locs, w[:1], mu[:1], cov[:1])
    np.testing.assert_allclose(E1, mu[0, 3], rtol=1e-14)
    np.testing.assert_allclose(V1, cov[0, 3, 3], rtol=1e-12)


# ------------------------------------------------------------ joint sampling

def test_sample_component_picks_match_exact_running_sum():
    w = np.random.default_rng(3).uniform(0.01, 1.0, 37).astype(np.float32).astype(np.float64)
    mu = np.zeros((37, 4))
    cov = np.tile(np.eye(4), (37, 1, 1))
    u = np.random.default_rng(4).random(5000)
    u[:3] = [0.0, 1.0 - 2.0 ** -53, 0.5]
    _, comp = gmm4.joint_sample(w, mu, cov, u, np.zeros((5000, 4)))
    wq = [Fraction(float(v)) for v in w]
    W = sum(wq)
    run = np.cumsum([float(v) for v in wq])  # for locating only
    for s in range(5000):
        t = Fraction(float(u[s])) * W
        acc, b = Fraction(0), 0
        for b, v in enumerate(wq):
            acc += v
            if acc > t:
                break
        # the exact pick; the oracle may differ only within rounding of the
        # running sum, which does not happen on these draws
        assert comp[s] == b, (s, comp[s], b)
    assert comp[0] == 0 and comp[1] == 36
    assert run[-1] > 0


def test_single_component_identity_sample_is_mean_plus_z():
    rng = np.random.default_rng(9)
    z = rng.standard_normal((100, 4))
    mu = np.array([[1.0, -2.0, 0.5, 0.25]])
    out, comp = gmm4.joint_sample([1.0], mu, np.eye(4)[None], rng.random(100), z)
    np.testing.assert_array_equal(out, mu + z)
    assert not comp.any()


def test_sample_moments_match_the_mixture():
    """400,000 draws: component frequencies within 5 binomial standard
    deviations of pi, the sample mean and covariance of each component
    within 5 standard errors of mu_b and Sigma_b."""
    w, mu, cov = _theta4(3, 11, spread=3.0)
    M = 400_000
    rng = np.random.default_rng(12)
    out, comp = gmm4.joint_sample(w, mu, cov, rng.random(M), rng.standard_normal((M, 4)))
    freq = np.bincount(comp, minlength=3) / M
    assert np.all(np.abs(freq - w) <= 5 * np.sqrt(w * (1 - w) / M)), (freq, w)
    for b in range(3):
        Y = out[comp == b]
        n = Y.shape[0]
        se = np.sqrt(np.diag(cov[b]) / n)
        assert np.all(np.abs(Y.mean(axis=0) - mu[b]) <= 5 * se)
        C = np.cov(Y.T)
        sd = np.sqrt((cov[b] ** 2 + np.outer(np.diag(cov[b]), np.diag(cov[b]))) / n)
        assert np.all(np.abs(C - cov[b]) <= 5 * sd)


def test_model_size_formula():
    """4 bytes x M x (1 + 4 + 10) for a 4D model: 69.78 kB is M = 1163."""
    M = 1163
    w, mu, cov = np.zeros(M, np.float32), np.zeros((M, 4), np.float32), np.zeros((M, 4, 4))
    tri = cov[:, np.tril_indices(4)[0], np.tril_indices(4)[1]].astype(np.float32)
    nbytes = w.nbytes + mu.nbytes + tri.nbytes
    assert nbytes == 4 * M * (1 + 10 + 4) == 69780
