"""FP64 oracle of the 4D mixture model (x, y, z, intensity): EM fitting,
conditional intensity and joint sampling.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers; nothing in the HIP
library imports, links or runs this module, and it uses nothing of the HIP
library.  Plain numpy in double precision, one component at a time, written
for any dimension D (the paper's model has D = 4).

What is computed (the paper, Sec. IV "GIRA Reconstruction" and Sec. V
"Expectation Maximization"):

* The model is a D = 4 Gaussian mixture over a point and its intensity:
  weights (K), means (K, 4), covariances (K, 4, 4); its size is 4 bytes x
  K x (1 + 4 + 10) (a symmetric 4 x 4 covariance has 10 free values).
* EM: E-step eq. 1-3 (responsibilities in the log domain from the
  Cholesky precision factor P_b = chol(Sigma_b)^-1:
  ln N(x | mu_b, Sigma_b) = -1/2 (D ln 2pi + |P_b (x - mu_b)|^2)
  + sum_j ln (P_b)_jj); the M-step is the standard maximum-likelihood
  update of full covariances (the paper names it, prints no formula), with
  the same conventions as the 3D fit: N_b = sum gamma + 10 DBL_EPSILON,
  pi_b = N_b / sum_a N_a, two-pass centred scatter, lambda on the diagonal.
* Conditional intensity ("color_conditional" in the paper's interface):
  for a location x (3D), the intensity given x under the 4D mixture is a
  mixture of 1D Gaussians with weights beta_b(x) proportional to
  pi_b N(x | mu_b^x, Sigma_b^xx) (the 3D marginals), means
  m_b(x) = mu_b^i + Sigma_b^ix (Sigma_b^xx)^-1 (x - mu_b^x) and variances
  v_b = Sigma_b^ii - Sigma_b^ix (Sigma_b^xx)^-1 Sigma_b^xi (Gaussian
  conditioning); E = sum_b beta_b m_b and V = sum_b beta_b (v_b + m_b^2)
  - E^2 (the variance of that conditional mixture).
* Joint sampling ("joint_dist_sample"): for each sample a component b with
  probability pi_b / sum_a pi_a, then mu_b + chol(Sigma_b) z with z a
  standard normal D-vector.  The draws are inputs: u (M uniforms in
  [0, 1)) picks the first component whose running sum of the weights (in
  component order, double precision) exceeds u sum_a pi_a; z (M x D).
"""
from __future__ import annotations

import numpy as np

EPS_N = 10.0 * np.finfo(np.float64).eps
LN2PI = float(np.log(2.0 * np.pi))


def _theta(w, mu, cov):
    w = np.asarray(w, np.float64).reshape(-1)
    K = w.shape[0]
    mu = np.asarray(mu, np.float64).reshape(K, -1)
    D = mu.shape[1]
    cov = np.asarray(cov, np.float64).reshape(K, D, D)
    return w, mu, cov, K, D


def component_terms(w, cov):
    """Eq. 3 terms per component: P_b = L_b^-1 with Sigma_b = L_b L_b^T, and
    c_b = ln pi_b - D/2 ln 2pi + sum_j ln (P_b)_jj.  A covariance that is not
    positive definite raises LinAlgError."""
    w = np.asarray(w, np.float64).reshape(-1)
    cov = np.asarray(cov, np.float64)
    K, D = cov.shape[0], cov.shape[1]
    P = np.zeros((K, D, D))
    c = np.zeros(K)
    for b in range(K):
        Sb = np.tril(cov[b]) + np.tril(cov[b], -1).T      # lower triangle read
        L = np.linalg.cholesky(Sb)
        P[b] = np.linalg.inv(L)
        P[b] = np.tril(P[b])
        c[b] = np.log(w[b]) - 0.5 * D * LN2PI + np.log(np.diag(P[b])).sum()
    return P, c


def log_terms(X, w, mu, cov):
    """l_nb = ln pi_b + ln N(x_n | mu_b, Sigma_b) (eq. 3), shape (N, K)."""
    w, mu, cov, K, D = _theta(w, mu, cov)
    X = np.asarray(X, np.float64).reshape(-1, D)
    P, c = component_terms(w, cov)
    l = np.empty((X.shape[0], K))
    for b in range(K):
        z = (X - mu[b]) @ P[b].T
        l[:, b] = c[b] - 0.5 * (z * z).sum(axis=1)
    return l


def estep(X, w, mu, cov):
    """E-step (eq. 1-2): (L, lse (N,), gamma (N, K)); max-shifted
    log-sum-exp, L = sum_n lse_n in nats."""
    l = log_terms(X, w, mu, cov)
    m = l.max(axis=1)
    lse = m + np.log(np.exp(l - m[:, None]).sum(axis=1))
    gamma = np.exp(l - lse[:, None])
    return float(lse.sum()), lse, gamma


def mstep(X, gamma, reg):
    """M-step from responsibilities (N, K): exact two-pass centring."""
    X = np.asarray(X, np.float64)
    N, D = X.shape
    K = gamma.shape[1]
    Nb = gamma.sum(axis=0) + EPS_N
    w = Nb / Nb.sum()
    mu = (gamma.T @ X) / Nb[:, None]
    cov = np.empty((K, D, D))
    for b in range(K):
        d = X - mu[b]
        cov[b] = (gamma[:, b, None] * d).T @ d / Nb[b] + reg * np.eye(D)
    return w, mu, cov


def mstep_labels(X, labels, K, reg):
    """M-step of the one-hot responsibilities of hard labels."""
    X = np.asarray(X, np.float64)
    g = np.zeros((X.shape[0], K))
    g[np.arange(X.shape[0]), np.asarray(labels)] = 1.0
    return mstep(X, g, reg)


def em_step(X, w, mu, cov, reg):
    """One EM iteration from theta: (w', mu', cov', L(theta))."""
    L, _, g = estep(X, w, mu, cov)
    return (*mstep(X, g, reg), L)


def fit(X, K, reg, iters, labels=None, theta0=None):
    """Fixed-iteration EM from hard labels (theta_0 = their M-step) or from
    theta0; returns (w, mu, cov, L history of iters + 1 values), the last
    L evaluated at the returned parameters."""
    X = np.asarray(X, np.float64)
    if labels is not None:
        w, mu, cov = mstep_labels(X, labels, K, reg)
    else:
        w, mu, cov, _, _ = _theta(*theta0)
    Lh = np.empty(iters + 1)
    for t in range(iters):
        w, mu, cov, Lh[t] = em_step(X, w, mu, cov, reg)
    Lh[iters] = estep(X, w, mu, cov)[0]
    return w, mu, cov, Lh


def color_conditional(locs, w, mu, cov):
    """Expected intensity and its variance at 3D locations under a 4D
    mixture (the conditional distribution of the last coordinate given the
    first three).  Returns (E (M,), V (M,), beta (M, K))."""
    w, mu, cov, K, D = _theta(w, mu, cov)
    assert D == 4
    locs = np.asarray(locs, np.float64).reshape(-1, 3)
    M = locs.shape[0]
    lb = np.empty((M, K))
    mb = np.empty((M, K))
    vb = np.empty(K)
    for b in range(K):
        S = np.tril(cov[b]) + np.tril(cov[b], -1).T
        Sxx, Sxi, Sii = S[:3, :3], S[:3, 3], S[3, 3]
        Lx = np.linalg.cholesky(Sxx)
        z = np.linalg.solve(Lx, (locs - mu[b, :3]).T).T      # Lx^-1 (x - mu)
        lb[:, b] = (np.log(w[b]) - 1.5 * LN2PI - np.log(np.diag(Lx)).sum()
                    - 0.5 * (z * z).sum(axis=1))
        A = np.linalg.solve(Sxx, Sxi)                          # Sxx^-1 Sxi
        mb[:, b] = mu[b, 3] + (locs - mu[b, :3]) @ A
        vb[b] = Sii - Sxi @ A
    m = lb.max(axis=1)
    beta = np.exp(lb - m[:, None])
    beta /= beta.sum(axis=1, keepdims=True)
    E = (beta * mb).sum(axis=1)
    V = (beta * (vb[None, :] + mb * mb)).sum(axis=1) - E * E
    return E, V, beta


def joint_sample(w, mu, cov, u, z):
    """Samples of the mixture from given draws: component of sample s = the
    first b whose running sum pi_0 + ... + pi_b (double, component order)
    exceeds u_s W, W the total (the last component with pi > 0 when
    rounding leaves none); sample = mu_b + chol(Sigma_b) z_s.  Returns
    (samples (M, D), components (M,) int64)."""
    w, mu, cov, K, D = _theta(w, mu, cov)
    u = np.asarray(u, np.float64).reshape(-1)
    z = np.asarray(z, np.float64).reshape(u.shape[0], D)
    run = np.empty(K)
    acc = 0.0
    for b in range(K):
        acc += w[b]
        run[b] = acc
    W = run[-1]
    last = int(np.flatnonzero(w > 0)[-1])
    comp = np.empty(u.shape[0], np.int64)
    for s in range(u.shape[0]):
        t = u[s] * W
        b = int(np.searchsorted(run, t, side="right"))   # first run[b] > t
        comp[s] = min(b, last) if b < K else last
    L = np.stack([np.linalg.cholesky(np.tril(c) + np.tril(c, -1).T) for c in cov])
    out = mu[comp] + np.einsum("sij,sj->si", L[comp], z)
    return out, comp
