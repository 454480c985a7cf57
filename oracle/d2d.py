"""FP64 oracle of distribution-to-distribution (D2D) registration of two
Gaussian mixtures.

TEST INFRASTRUCTURE ONLY.  The test suite and the benchmark's CPU-baseline
leg are the only callers; nothing in the HIP library imports or runs this
module, and it uses nothing of the HIP library.  Plain numpy in double
precision, one component pair at a time where it matters.

The paper (Sec. IV "GIRA Registration") registers a source mixture to a
target mixture with the anisotropic, isoplanar and isoplanar-then-
anisotropic variants of its cited on-manifold GMM registration, returning
the SE(3) transform; it gives no formulas.  The readings taken here:

  objective   f(T) = ln sum_ij pi_i tau_j N(R mu_i + t; nu_j, R Sigma_i R^T
              + Lambda_j), the log of the integral of the product of the
              transformed source density and the target density (a
              Gaussian product integrates in closed form), maximised over
              T = (R, t);
  variants    anisotropic: the mixtures' own covariances; isoplanar: every
              covariance replaced by V diag(1, 1, eps) V^T with V its
              eigenvectors by decreasing eigenvalue and eps = 1e-3 (a plane
              through the component with unit in-plane variance), i.e.
              I - (1 - eps) v v^T for v the eigenvector of the smallest
              eigenvalue; hybrid: isoplanar iterations, then anisotropic
              ones from the result;
  step        a Newton-type ascent step in the left-perturbation
              coordinates (delta, dt): the curvature is the Gauss-Newton
              matrix of the EM lower bound of f (gamma_ij = the pair's share
              of the sum at T, S_ij held at T, residual d_ij = R mu_i + t -
              nu_j, J_ij = [-[R mu_i]_x, I], H = sum gamma J^T S^-1 J), the
              right-hand side is the exact gradient (so that the steps stop
              where f is stationary: with S held fixed the rotation of the
              covariances would be left out), x = H^-1 grad f (FP64
              Cholesky); trial poses
              R' = exp([s x_w]_x) R, t' = t + s x_t for s = 1, 1/2, ...,
              2^-7; the first trial with f(T') > f(T) is taken; the stage
              ends when max|x| < 1e-8, when H is not positive definite,
              when no trial increases f, or after its iteration budget.

The pose enters as (omega, t) with R = exp([omega]_x) (Rodrigues) and leaves
as the 4 x 4 transform.  Gradients are with respect to (omega, t): a left
perturbation delta of R gives df/d delta, and df/d omega = J_l(omega)^T
df/d delta with J_l the left Jacobian of SO(3).
"""
from __future__ import annotations

import numpy as np

LN2PI = np.log(2.0 * np.pi)
ISO_EPS = 1e-3
N_TRIALS = 8
STEP_TOL = 1e-8


def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def expso3(w):
    """Rodrigues' formula (series below |w| = 1e-4)."""
    w = np.asarray(w, np.float64)
    th = float(np.sqrt(w @ w))
    K = skew(w)
    if th < 1e-4:
        a = 1.0 - th * th / 6.0
        b = 0.5 - th * th / 24.0
    else:
        a = np.sin(th) / th
        b = (1.0 - np.cos(th)) / (th * th)
    return np.eye(3) + a * K + b * (K @ K)


def left_jacobian(w):
    w = np.asarray(w, np.float64)
    th = float(np.sqrt(w @ w))
    K = skew(w)
    if th < 1e-4:
        a = 0.5 - th * th / 24.0
        b = 1.0 / 6.0 - th * th / 120.0
    else:
        a = (1.0 - np.cos(th)) / (th * th)
        b = (th - np.sin(th)) / (th ** 3)
    return np.eye(3) + a * K + b * (K @ K)


def isoplanar(cov):
    """V diag(1, 1, eps) V^T for each covariance (eigh: ascending order, so
    the first eigenvector is the normal)."""
    cov = np.asarray(cov, np.float64)
    out = np.empty_like(cov)
    for k in range(cov.shape[0]):
        _, V = np.linalg.eigh(cov[k])
        v = V[:, 0]
        out[k] = np.eye(3) - (1.0 - ISO_EPS) * np.outer(v, v)
    return out


def pair_terms(R, t, src, tgt):
    """l_ij, and per pair (a_i = R mu_i, S_ij, d_ij, Sigma'_i) for the
    gradient: a list of dicts would be slow, so arrays (M, N, ...)."""
    w, mu, cov = src
    tw, tmu, tcov = tgt
    a = mu @ R.T                                   # R mu_i
    Sp = np.einsum("ab,ibc,dc->iad", R, cov, R)    # R Sigma_i R^T
    S = Sp[:, None] + tcov[None]                   # (M, N, 3, 3)
    d = (a + t)[:, None] - tmu[None]               # (M, N, 3)
    L = np.linalg.cholesky(S)
    logdet = 2.0 * np.log(np.diagonal(L, axis1=-2, axis2=-1)).sum(-1)
    g = np.linalg.solve(S, d[..., None])[..., 0]   # S^-1 d
    quad = np.einsum("ija,ija->ij", d, g)
    ell = (np.log(w)[:, None] + np.log(tw)[None] - 1.5 * LN2PI - 0.5 * logdet
           - 0.5 * quad)
    return ell, a, S, d, g, Sp


def _lse(ell):
    m = ell.max()
    return float(m + np.log(np.exp(ell - m).sum()))


def objective(pose6, src, tgt):
    """f(T) for pose6 = (omega, t)."""
    R = expso3(pose6[:3])
    ell = pair_terms(R, np.asarray(pose6[3:], np.float64), src, tgt)[0]
    return _lse(ell)


def grad_delta(R, t, src, tgt):
    """(f, df/d(delta, dt)) for a left perturbation exp([delta]_x) R of R
    and t + dt."""
    ell, a, S, d, g, Sp = pair_terms(R, t, src, tgt)
    f = _lse(ell)
    gam = np.exp(ell - f)
    # dl/dt = -g; dl/d delta = g x a + (A_23, A_31, A_12), A = Sigma' M - M Sigma',
    # M = g g^T - S^-1 (left perturbation of R)
    Sinv = np.linalg.inv(S)
    M = g[..., :, None] * g[..., None, :] - Sinv
    Spb = np.broadcast_to(Sp[:, None], S.shape)
    A = Spb @ M - M @ Spb
    ab = np.broadcast_to(a[:, None], d.shape)
    dl_dd = np.cross(g, ab) + np.stack([A[..., 1, 2], A[..., 2, 0], A[..., 0, 1]], -1)
    gd = np.einsum("ij,ija->a", gam, dl_dd)
    gt = -np.einsum("ij,ija->a", gam, g)
    return f, np.concatenate([gd, gt])


def objective_grad(pose6, src, tgt):
    """(f, df/d(omega, t)) at pose6 = (omega, t)."""
    pose6 = np.asarray(pose6, np.float64)
    f, gdt = grad_delta(expso3(pose6[:3]), pose6[3:], src, tgt)
    gw = left_jacobian(pose6[:3]).T @ gdt[:3]
    return f, np.concatenate([gw, gdt[3:]])


def gn_system(R, t, src, tgt):
    """f, the Gauss-Newton matrix H (6 x 6) and its right-hand side
    b = sum gamma J^T S^-1 d at (R, t)."""
    ell, a, S, d, g, _ = pair_terms(R, t, src, tgt)
    f = _lse(ell)
    gam = np.exp(ell - f)
    Sinv = np.linalg.inv(S)
    M = ell.shape[0]
    J = np.empty((M, 3, 6))                        # d(d_ij)/d(delta, dt), per source i
    for i in range(M):
        J[i, :, :3] = -skew(a[i])
        J[i, :, 3:] = np.eye(3)
    JS = np.einsum("iak,ijab->ijkb", J, Sinv)      # J^T S^-1
    H = np.einsum("ij,ijkb,ibl->kl", gam, JS, J)
    b = np.einsum("ij,ijkb,ijb->k", gam, JS, d)
    return f, H, b


def register(T0, src, tgt, iters_iso=30, iters_aniso=30):
    """Isoplanar then anisotropic Gauss-Newton registration from the 4 x 4
    transform T0.  Returns (T 4 x 4, history: list of (stage, f) per accepted
    iteration (the start value of each stage first), iterations per
    stage)."""
    T0 = np.asarray(T0, np.float64)
    R, t = T0[:3, :3].copy(), T0[:3, 3].copy()
    src = tuple(np.asarray(x, np.float64) for x in src)
    tgt = tuple(np.asarray(x, np.float64) for x in tgt)
    stages = []
    if iters_iso > 0:
        stages.append(("iso", (src[0], src[1], isoplanar(src[2])),
                       (tgt[0], tgt[1], isoplanar(tgt[2])), iters_iso))
    if iters_aniso > 0:
        stages.append(("aniso", src, tgt, iters_aniso))
    hist, counts = [], []
    for name, s, g, n in stages:
        f = _lse(pair_terms(R, t, s, g)[0])
        hist.append((name, f))
        done = 0
        for _ in range(n):
            _, H, _ = gn_system(R, t, s, g)
            _, grad = grad_delta(R, t, s, g)
            try:
                Lc = np.linalg.cholesky(H)
            except np.linalg.LinAlgError:
                break
            x = np.linalg.solve(Lc.T, np.linalg.solve(Lc, grad))
            if np.abs(x).max() < STEP_TOL:
                break
            took = False
            for k in range(N_TRIALS):
                sc = 0.5 ** k
                R1 = expso3(sc * x[:3]) @ R
                t1 = t + sc * x[3:]
                f1 = _lse(pair_terms(R1, t1, s, g)[0])
                if f1 > f:
                    R, t, f, took = R1, t1, f1, True
                    break
            if not took:
                break
            done += 1
            hist.append((name, f))
        counts.append(done)
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T, hist, counts
