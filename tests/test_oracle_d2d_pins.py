"""Pins of the D2D registration oracle (oracle/d2d.py) against things other
than itself:

* one component on each side: f is the log density of a Gaussian at the
  transformed mean (scipy's multivariate_normal as a black box);
* the closed form of the objective against the integral it stands for (the
  product of the two densities integrated on a 3D grid);
* the gradient against central finite differences of f and against torch
  FP64 autograd of an independent expression (matrix exponential of the
  skew matrix, torch.logsumexp, MultivariateNormal.log_prob);
* Cauchy-Schwarz: for a mixture against itself the identity is the global
  maximum (f(T) <= f(I), gradient zero at I), and a mixture against a
  rigidly moved copy of itself is maximised at that motion, which the
  registration recovers from a nearby start;
* isoplanar covariances have eigenvalues (1, 1, 1e-3) about the smallest
  eigenvector of the original;
* the Gauss-Newton right-hand side's translation part is minus the
  gradient's, and its rotation part differs from minus the rotation
  gradient exactly by the covariance-rotation term (zero for isotropic
  covariances).
"""
import numpy as np
import pytest

from oracle import d2d


def _mixture(seed, m, spread=1.5, smin=0.05, smax=0.4):
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, m)
    w /= w.sum()
    mu = rng.uniform(-spread, spread, (m, 3))
    cov = np.empty((m, 3, 3))
    for k in range(m):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q *= np.sign(np.diag(r))
        s = rng.uniform(smin, smax, 3)
        cov[k] = q @ np.diag(s * s) @ q.T
    return w, mu, cov


def _moved(mix, R, t):
    w, mu, cov = mix
    return w, mu @ R.T + t, np.einsum("ab,kbc,dc->kad", R, cov, R)


def test_single_components_are_a_gaussian_log_density():
    from scipy.stats import multivariate_normal
    src = _mixture(1, 1)
    tgt = _mixture(2, 1)
    pose = np.array([0.2, -0.1, 0.3, 0.05, 0.1, -0.2])
    R = d2d.expso3(pose[:3])
    S = R @ src[2][0] @ R.T + tgt[2][0]
    ref = (np.log(src[0][0]) + np.log(tgt[0][0]) +
           multivariate_normal(tgt[1][0], S).logpdf(R @ src[1][0] + pose[3:]))
    assert abs(d2d.objective(pose, src, tgt) - ref) <= 1e-12 * abs(ref)


def test_objective_is_the_product_integral():
    """ln of the grid integral of p_src,T(x) p_tgt(x) (two components each,
    broad enough for a 161^3 grid over +-4 m to resolve)."""
    from scipy.stats import multivariate_normal
    src = _mixture(3, 2, spread=0.8, smin=0.4, smax=0.8)
    tgt = _mixture(4, 2, spread=0.8, smin=0.4, smax=0.8)
    pose = np.array([0.1, 0.2, -0.15, 0.1, -0.05, 0.2])
    R = d2d.expso3(pose[:3])
    ms = _moved(src, R, pose[3:])
    g = np.linspace(-4, 4, 161)
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    ps = sum(ms[0][k] * multivariate_normal(ms[1][k], ms[2][k]).pdf(X) for k in range(2))
    pt = sum(tgt[0][k] * multivariate_normal(tgt[1][k], tgt[2][k]).pdf(X) for k in range(2))
    integral = (ps * pt).sum() * (g[1] - g[0]) ** 3
    assert abs(d2d.objective(pose, src, tgt) - np.log(integral)) <= 1e-6


@pytest.mark.parametrize("seed", [5, 6])
def test_gradient_matches_finite_differences(seed):
    src = _mixture(seed, 7)
    tgt = _mixture(seed + 100, 9)
    pose = np.array([0.3, -0.2, 0.1, 0.2, 0.1, -0.1])
    f, g = d2d.objective_grad(pose, src, tgt)
    assert abs(f - d2d.objective(pose, src, tgt)) <= 1e-13 * abs(f)
    h = 1e-6
    fd = np.empty(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        fd[k] = (d2d.objective(pose + e, src, tgt) - d2d.objective(pose - e, src, tgt)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    src = _mixture(8, 5)
    tgt = _mixture(9, 6)
    pose = np.array([-0.25, 0.15, 0.35, -0.3, 0.2, 0.05])
    p = torch.tensor(pose, dtype=torch.float64, requires_grad=True)
    w = p[:3]
    K = torch.zeros(3, 3, dtype=torch.float64)
    K = K.index_put((torch.tensor([0, 0, 1, 1, 2, 2]), torch.tensor([1, 2, 0, 2, 0, 1])),
                    torch.stack([-w[2], w[1], w[2], -w[0], -w[1], w[0]]))
    R = torch.linalg.matrix_exp(K)
    mu = torch.tensor(src[1]) @ R.T + p[3:]
    cov = R @ torch.tensor(src[2]) @ R.T
    terms = []
    for i in range(5):
        for j in range(6):
            S = cov[i] + torch.tensor(tgt[2][j])
            dist = torch.distributions.MultivariateNormal(torch.tensor(tgt[1][j]), S)
            terms.append(np.log(src[0][i]) + np.log(tgt[0][j]) + dist.log_prob(mu[i]))
    f = torch.logsumexp(torch.stack(terms), 0)
    f.backward()
    fo, go = d2d.objective_grad(pose, src, tgt)
    assert abs(fo - f.item()) <= 1e-12 * abs(fo)
    np.testing.assert_allclose(go, p.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_self_registration_maximum_at_identity():
    mix = _mixture(10, 8)
    f0, g0 = d2d.objective_grad(np.zeros(6), mix, mix)
    assert np.abs(g0).max() <= 1e-9 * max(1.0, abs(f0))
    rng = np.random.default_rng(11)
    for _ in range(10):
        pose = rng.normal(0, 0.2, 6)
        assert d2d.objective(pose, mix, mix) < f0


@pytest.mark.parametrize("iso", [0, 20])
def test_register_recovers_a_rigid_motion(iso):
    """tgt = src moved by (R*, t*): the objective peaks at T* (Cauchy-
    Schwarz); from the identity the registration reaches it (a hybrid run
    and a purely anisotropic one)."""
    src = _mixture(12, 10)
    Rs = d2d.expso3(np.array([0.15, -0.1, 0.2]))
    ts = np.array([0.2, -0.1, 0.15])
    tgt = _moved(src, Rs, ts)
    T, hist, counts = d2d.register(np.eye(4), src, tgt, iters_iso=iso, iters_aniso=40)
    np.testing.assert_allclose(T[:3, :3], Rs, atol=1e-7)
    np.testing.assert_allclose(T[:3, 3], ts, atol=1e-7)
    fs = [f for st, f in hist if st == "aniso"]
    assert all(b > a for a, b in zip(fs, fs[1:]))   # every accepted step increases f
    assert counts[-1] >= 1


def test_isoplanar_covariances():
    cov = np.array([np.diag([3.0, 2.0, 0.1]), np.diag([0.2, 5.0, 1.0])])
    iso = d2d.isoplanar(cov)
    np.testing.assert_allclose(iso[0], np.diag([1.0, 1.0, 1e-3]), atol=1e-15)
    np.testing.assert_allclose(iso[1], np.diag([1e-3, 1.0, 1.0]), atol=1e-15)
    _, _, c = _mixture(13, 4)
    iso = d2d.isoplanar(c)
    for k in range(4):
        ev, V = np.linalg.eigh(c[k])
        ei = np.linalg.eigvalsh(iso[k])
        np.testing.assert_allclose(ei, [1e-3, 1.0, 1.0], atol=1e-14)
        np.testing.assert_allclose(iso[k] @ V[:, 0], 1e-3 * V[:, 0], atol=1e-14)


def test_gauss_newton_rhs_translation_is_minus_the_gradient():
    src = _mixture(14, 6)
    tgt = _mixture(15, 7)
    pose = np.array([0.1, 0.0, -0.2, 0.3, -0.1, 0.2])
    f, g = d2d.objective_grad(pose, src, tgt)
    R = d2d.expso3(pose[:3])
    f2, H, b = d2d.gn_system(R, pose[3:], src, tgt)
    assert abs(f - f2) <= 1e-13 * abs(f)
    np.testing.assert_allclose(b[3:], -g[3:], rtol=1e-12, atol=1e-14)
    assert np.all(np.linalg.eigvalsh(H) > 0)
    # isotropic covariances: no covariance-rotation term, b = -grad exactly
    iso_src = (src[0], src[1], np.stack([np.eye(3) * 0.04] * 6))
    iso_tgt = (tgt[0], tgt[1], np.stack([np.eye(3) * 0.09] * 7))
    _, gd = d2d.grad_delta(R, pose[3:], iso_src, iso_tgt)
    _, _, b2 = d2d.gn_system(R, pose[3:], iso_src, iso_tgt)
    np.testing.assert_allclose(b2, -gd, rtol=1e-10, atol=1e-12 * np.abs(gd).max())
