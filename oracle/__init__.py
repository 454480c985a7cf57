"""FP64 CPU oracle for GMM EM fitting and the GMM registration log-likelihood.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers; the HIP library never
imports, links or runs anything here, and this package never touches the
HIP library.  The arithmetic lives in ``gmm_oracle.c`` (plain C, double
precision); this module only marshals numpy arrays to it.

Functions follow the paper's Sec. V "Expectation Maximization":
eq. 1 (responsibilities), eq. 2 (log-domain E-step), eq. 3 (Cholesky
precision form of the Gaussian log-density); the M-step is the standard
full-covariance maximum-likelihood update (the paper names it without
formulas).  ``kmeanspp`` is the k-means++ seeding read into the randomised
k-means initialisation that precedes EM in the same section (its draws are
inputs; the draw is turned into an index by one flat running sum).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "ok", 1: "invalid argument", 2: "covariance not SPD",
          3: "non-finite result", 4: "out of memory"}


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        D = ctypes.POINTER(ctypes.c_double)
        I32 = ctypes.POINTER(ctypes.c_int32)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.oracle_set_threads.argtypes = [i32]
        lib.oracle_get_threads.restype = i32
        lib.oracle_component_terms.argtypes = [i32, D, D, D, D]
        lib.oracle_estep.argtypes = [i64, D, i32, D, D, D, D, D, D]
        lib.oracle_mstep_labels.argtypes = [i64, D, I32, i32, dbl, D, D, D]
        lib.oracle_em_step.argtypes = [i64, D, i32, D, D, D, dbl, D, D, D, D]
        lib.oracle_fit.argtypes = [i64, D, i32, I32, D, D, D, dbl, i32, D]
        lib.oracle_loglik_pose.argtypes = [i64, D, D, i32, D, D, D, D, D]
        lib.oracle_loglik_grad.argtypes = [i64, D, D, i32, D, D, D, dbl,
                                           D, D, D, D, D]
        lib.oracle_kmeanspp.argtypes = [i64, D, i32, D,
                                        ctypes.POINTER(ctypes.c_int64), I32]
        lib.oracle_nearest.argtypes = [i64, D, i32, ctypes.POINTER(ctypes.c_int64),
                                       I32]
        lib.oracle_kmeanspp_replay.argtypes = [
            i64, D, i32, D, ctypes.POINTER(ctypes.c_int64),
            ctypes.POINTER(ctypes.c_int64), D, D, D]
        for name in ("oracle_kmeanspp_replay", "oracle_nearest", "oracle_component_terms", "oracle_estep",
                     "oracle_mstep_labels", "oracle_em_step", "oracle_fit",
                     "oracle_loglik_pose", "oracle_loglik_grad",
                     "oracle_kmeanspp"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _check(st):
    if st != 0:
        raise OracleError(STATUS.get(st, "status %d" % st))


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def component_terms(w, cov):
    """Eq. 3 terms: precision Cholesky P_b = chol(Sigma_b)^-1 (K,3,3) and
    c_b = ln pi_b - 3/2 ln 2pi + sum_j ln P_b,jj (K,)."""
    w = _f64(w)
    K = w.shape[0]
    cov = _f64(cov, (K, 3, 3))
    P = np.zeros((K, 3, 3))
    c = np.zeros(K)
    _check(_load().oracle_component_terms(K, _d(w), _d(cov), _d(P), _d(c)))
    return P, c


def estep(X, w, mu, cov, want_lse=True, want_logresp=False):
    """E-step (eq. 1-3): returns (L, lse_n or None, ln gamma (N,K) or None)."""
    X = _f64(X)
    X = X.reshape(-1, 3)
    w = _f64(w)
    K = w.shape[0]
    mu = _f64(mu, (K, 3))
    cov = _f64(cov, (K, 3, 3))
    N = X.shape[0]
    lse = np.zeros(N) if want_lse else None
    lr = np.zeros((N, K)) if want_logresp else None
    L = ctypes.c_double(0.0)
    _check(_load().oracle_estep(N, _d(X), K, _d(w), _d(mu), _d(cov), _d(lse),
                                _d(lr), ctypes.byref(L)))
    return L.value, lse, lr


def mstep_labels(X, labels, K, reg):
    """M-step of the one-hot responsibilities given by hard labels."""
    X = _f64(X).reshape(-1, 3)
    lab = np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
    w = np.zeros(K)
    mu = np.zeros((K, 3))
    cov = np.zeros((K, 3, 3))
    _check(_load().oracle_mstep_labels(
        X.shape[0], _d(X), lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        K, float(reg), _d(w), _d(mu), _d(cov)))
    return w, mu, cov


def em_step(X, w, mu, cov, reg):
    """One EM iteration from theta: returns (w', mu', cov', L(theta))."""
    X = _f64(X).reshape(-1, 3)
    w = _f64(w)
    K = w.shape[0]
    mu = _f64(mu, (K, 3))
    cov = _f64(cov, (K, 3, 3))
    wo, muo, covo = np.zeros(K), np.zeros((K, 3)), np.zeros((K, 3, 3))
    L = ctypes.c_double(0.0)
    _check(_load().oracle_em_step(X.shape[0], _d(X), K, _d(w), _d(mu), _d(cov),
                                  float(reg), _d(wo), _d(muo), _d(covo),
                                  ctypes.byref(L)))
    return wo, muo, covo, L.value


def fit(X, K, reg, iters, labels=None, theta0=None):
    """Fixed-iteration EM.  Start from hard labels (theta_0 = their M-step)
    or from theta0 = (w, mu, cov).  Returns (w, mu, cov, Lhist[T+1])."""
    X = _f64(X).reshape(-1, 3)
    if labels is not None:
        lab = np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
        labp = lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        w, mu, cov = np.zeros(K), np.zeros((K, 3)), np.zeros((K, 3, 3))
    else:
        labp = None
        w = _f64(theta0[0]).copy()
        mu = _f64(theta0[1], (K, 3)).copy()
        cov = _f64(theta0[2], (K, 3, 3)).copy()
    Lh = np.zeros(iters + 1)
    _check(_load().oracle_fit(X.shape[0], _d(X), K, labp, _d(w), _d(mu),
                              _d(cov), float(reg), int(iters), _d(Lh)))
    return w, mu, cov, Lh


def loglik_pose(X, pose6, w, mu, cov, want_lse=False):
    """L(pose) = sum_n lse_n(R(omega) x_n + t); pose6 None = identity."""
    X = _f64(X).reshape(-1, 3)
    w = _f64(w)
    K = w.shape[0]
    mu = _f64(mu, (K, 3))
    cov = _f64(cov, (K, 3, 3))
    p = None if pose6 is None else _f64(pose6, (6,))
    lse = np.zeros(X.shape[0]) if want_lse else None
    L = ctypes.c_double(0.0)
    _check(_load().oracle_loglik_pose(X.shape[0], _d(X), _d(p), K, _d(w),
                                      _d(mu), _d(cov), ctypes.byref(L), _d(lse)))
    return (L.value, lse) if want_lse else L.value


def loglik_grad(X, pose6, w, mu, cov, grad_L=1.0):
    """Analytic gradient of grad_L * L(pose, X, w, mu, cov).
    Returns dict with pose (6,), pts (N,3), w (K,), mu (K,3), cov (K,3,3)."""
    X = _f64(X).reshape(-1, 3)
    w = _f64(w)
    K = w.shape[0]
    mu = _f64(mu, (K, 3))
    cov = _f64(cov, (K, 3, 3))
    p = None if pose6 is None else _f64(pose6, (6,))
    out = dict(pose=np.zeros(6), pts=np.zeros_like(X), w=np.zeros(K),
               mu=np.zeros((K, 3)), cov=np.zeros((K, 3, 3)))
    _check(_load().oracle_loglik_grad(
        X.shape[0], _d(X), _d(p), K, _d(w), _d(mu), _d(cov), float(grad_L),
        _d(out["pose"]), _d(out["pts"]), _d(out["w"]), _d(out["mu"]),
        _d(out["cov"])))
    return out


def kmeanspp(X, K, u):
    """k-means++ D^2 seeding with the K uniform draws u (in [0, 1)) given,
    and nearest-seed labels (ties to the lowest index).  Returns
    (centre indices int64 (K,), labels int32 (N,)).  Centre j >= 1 is the
    first index whose flat running sum of D^2 (in index order, double
    precision) exceeds u[j] * W; see oracle_kmeanspp in gmm_oracle.c."""
    X = _f64(X).reshape(-1, 3)
    u = _f64(u)
    K = int(K)
    if u.shape != (K,):
        raise OracleError("need K uniform draws")
    N = X.shape[0]
    cen = np.zeros(K, dtype=np.int64)
    lab = np.zeros(N, dtype=np.int32)
    _check(_load().oracle_kmeanspp(
        N, _d(X), K, _d(u), cen.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return cen, lab


def nearest(X, centres):
    """Hard labels: for each point the index j of the nearest centre
    X[centres[j]] (squared distance ((dx^2 + dy^2) + dz^2) in double, the
    lowest j on ties).  Returns int32 (N,)."""
    X = _f64(X).reshape(-1, 3)
    cen = np.ascontiguousarray(np.asarray(centres, dtype=np.int64))
    lab = np.zeros(X.shape[0], dtype=np.int32)
    _check(_load().oracle_nearest(
        X.shape[0], _d(X), int(cen.shape[0]),
        cen.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return lab


def kmeanspp_replay(X, u, centres):
    """Replays the seeding `centres` (K indices) with draws u: per step j the
    flat running-sum pick on that trajectory (int64 (K,)), and the total W
    and the running sums before and at centres[j] as double-double (hi, lo)
    pairs (three float64 (K, 2) arrays; row 0 unused)."""
    X = _f64(X).reshape(-1, 3)
    u = _f64(u)
    cen = np.ascontiguousarray(np.asarray(centres, dtype=np.int64))
    K = int(cen.shape[0])
    if u.shape != (K,):
        raise OracleError("need K uniform draws")
    flat = np.zeros(K, dtype=np.int64)
    W, lo, at = np.zeros((K, 2)), np.zeros((K, 2)), np.zeros((K, 2))
    p64 = ctypes.POINTER(ctypes.c_int64)
    _check(_load().oracle_kmeanspp_replay(
        X.shape[0], _d(X), K, _d(u), cen.ctypes.data_as(p64),
        flat.ctypes.data_as(p64), _d(W), _d(lo), _d(at)))
    return flat, W, lo, at
