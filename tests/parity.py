"""Error measures of a GPU mixture against the FP64 oracle's.

Per parameter array A in {pi, mu, Sigma}: ||A_gpu - A_ref||_F / ||A_ref||_F.
Per component b with pi_b >= 1e-3 (a component that carries a visible share
of the points), so that an error confined to one thin component is not
hidden by the large ones:
  pi_b:     |dpi_b| / pi_b
  mu_b:     |dmu_b| / (|mu_b| + R), R the cloud's RMS radius about its mean
            (a mean error is measured against the scale of the scene);
  Sigma_b:  ||dSigma_b||_F / ||Sigma_b||_F.
"""
import numpy as np

PI_MIN = 1e-3


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rms_radius(X):
    X = np.asarray(X, np.float64)
    X = X.reshape(X.shape[0], -1)
    return float(np.sqrt(((X - X.mean(axis=0)) ** 2).sum(axis=1).mean()))


def per_component(got, ref, X, pi_min=PI_MIN):
    """Largest per-component errors over the components with pi_b >= pi_min
    (of the reference).  got / ref = (w, mu, cov)."""
    w, mu, cov = (np.asarray(a, np.float64) for a in got)
    wr, mur, covr = (np.asarray(a, np.float64) for a in ref)
    K = wr.shape[0]
    D = mur.size // K
    mu, mur = mu.reshape(K, D), mur.reshape(K, D)
    cov, covr = cov.reshape(K, D, D), covr.reshape(K, D, D)
    sel = wr >= pi_min
    if not sel.any():
        return {"pi_b": 0.0, "mu_b": 0.0, "cov_b": 0.0}
    R = rms_radius(X)
    e_pi = np.abs(w - wr)[sel] / wr[sel]
    e_mu = (np.linalg.norm(mu - mur, axis=1) /
            (np.linalg.norm(mur, axis=1) + R))[sel]
    e_cov = (np.linalg.norm((cov - covr).reshape(K, D * D), axis=1) /
             np.linalg.norm(covr.reshape(K, D * D), axis=1))[sel]
    return {"pi_b": float(e_pi.max()), "mu_b": float(e_mu.max()),
            "cov_b": float(e_cov.max())}


def mixture_errors(got, ref, X):
    """Array-wide and per-component errors in one dict."""
    e = {"w": rel(got[0], ref[0]), "mu": rel(got[1], ref[1]),
         "cov": rel(got[2], ref[2])}
    e.update(per_component(got, ref, X))
    return e


def elementwise(a, ref, rtol, atol_frac):
    """Largest |a - ref| / (rtol |ref| + atol_frac max|ref|) over all
    entries: <= 1 passes.  The absolute floor is a fraction of the array's
    largest magnitude, so entries that are sums of cancelling terms are
    judged on the array's scale."""
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = float(np.abs(ref).max()) if ref.size else 0.0
    den = rtol * np.abs(ref) + atol_frac * max(scale, 1e-300)
    return float((np.abs(a - ref) / den).max()) if ref.size else 0.0
