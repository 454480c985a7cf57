"""MI355X-native GMM EM fitting and differentiable GMM registration likelihood.

Thin PyTorch-facing layer over the HIP library ``libgmm.so`` (C ABI in
include/gmm.h).  PyTorch provides device memory and the current stream;
every arithmetic step runs in the library's kernels.

The method is the EM of GIRA (arXiv 2307.00071), Sec. V "Expectation
Maximization" (eq. 1-3), with the standard full-covariance M-step.
"""
from __future__ import annotations

import ctypes

from . import _lib

__all__ = ["fit", "fit_noalloc", "fit_batched", "loglik", "loglik_backward", "GMMLogLik",
           "FitResult", "kmeanspp", "fit4", "color_conditional", "joint_dist_sample",
           "meanshift", "d2d_objective", "d2d_register"]


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_points(points):
    torch = _torch()
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise TypeError("points must be a CUDA (HIP) torch tensor")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be float32 of shape (N, 3)")
    return points.contiguous()


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


class FitResult:
    """Parameters theta_T (float32) and the log-likelihood history (float64,
    iters + 1 entries, L(theta_t) in nats)."""

    def __init__(self, weights, means, covariances, loglik):
        self.weights = weights
        self.means = means
        self.covariances = covariances
        self.loglik = loglik

    def __iter__(self):
        return iter((self.weights, self.means, self.covariances, self.loglik))


def fit(points, k, iters=100, reg_covar=1e-3, labels=None, theta0=None,
        moment_mode="shifted", workspace=None, sync=True, tol=0.0):
    """EM fit of a K-component 3D GMM to ``points`` (float32 (N, 3), on GPU).

    Start either from hard ``labels`` (int32 (N,), values in [0, K)) whose
    one-hot M-step gives theta_0, or from ``theta0 = (w, mu, cov)``.
    ``tol`` > 0 stops early once the log-likelihood changes by at most
    tol * N between iterations (the skipped iterations' L entries are NaN)."""
    torch = _torch()
    lib = _lib.load()
    pts = _check_points(points)
    dev = pts.device
    n = pts.shape[0]
    opts = _lib.FitOpts(int(iters), float(reg_covar),
                        {"shifted": _lib.GMM_MOMENTS_SHIFTED,
                         "two_pass": _lib.GMM_MOMENTS_TWO_PASS}[moment_mode],
                        0 if sync else _lib.GMM_FLAG_ASYNC, float(tol))
    if labels is not None:
        lab = labels.to(device=dev, dtype=torch.int32).contiguous()
        if lab.shape != (n,):
            raise ValueError("labels must have shape (N,)")
        w = torch.empty(k, dtype=torch.float32, device=dev)
        mu = torch.empty(k, 3, dtype=torch.float32, device=dev)
        cov = torch.empty(k, 3, 3, dtype=torch.float32, device=dev)
    elif theta0 is not None:
        lab = None
        w = theta0[0].to(device=dev, dtype=torch.float32).contiguous().clone()
        mu = theta0[1].to(device=dev, dtype=torch.float32).contiguous().clone()
        cov = theta0[2].to(device=dev, dtype=torch.float32).contiguous().clone()
        if w.shape != (k,) or mu.shape != (k, 3) or cov.shape != (k, 3, 3):
            raise ValueError("theta0 shapes must be (K,), (K,3), (K,3,3)")
    else:
        raise ValueError("give labels or theta0")
    L = torch.empty(iters + 1, dtype=torch.float64, device=dev)
    need = lib.gmm_fit_workspace_size(n, k, ctypes.byref(opts))
    if need == 0:
        _lib.check(lib.gmm_fit(None, n, k, None, None, None, None, None,
                               ctypes.byref(opts), None, 0, None))
    ws = workspace if workspace is not None and workspace.numel() >= need \
        else _workspace(need, dev)
    st = lib.gmm_fit(_ptr(pts), n, k, _ptr(lab), _ptr(w), _ptr(mu), _ptr(cov),
                     _ptr(L), ctypes.byref(opts), _ptr(ws), ws.numel(),
                     _stream(dev))
    _lib.check(st)
    return FitResult(w, mu, cov, L)


def fit_noalloc(points, k, iters=100, reg_covar=1e-3, labels=None, theta0=None,
                moment_mode="shifted"):
    """``fit`` through gmm_fit_noalloc: the library allocates no device
    memory (its workspace is a fixed per-GPU array of
    GMM_FIT_NOALLOC_MAX_BYTES); the caller's tensors are the only buffers.
    Overlapping calls on one GPU race."""
    torch = _torch()
    lib = _lib.load()
    pts = _check_points(points)
    dev = pts.device
    n = pts.shape[0]
    opts = _lib.FitOpts(int(iters), float(reg_covar),
                        {"shifted": _lib.GMM_MOMENTS_SHIFTED,
                         "two_pass": _lib.GMM_MOMENTS_TWO_PASS}[moment_mode], 0)
    if labels is not None:
        lab = labels.to(device=dev, dtype=torch.int32).contiguous()
        if lab.shape != (n,):
            raise ValueError("labels must have shape (N,)")
        w = torch.empty(k, dtype=torch.float32, device=dev)
        mu = torch.empty(k, 3, dtype=torch.float32, device=dev)
        cov = torch.empty(k, 3, 3, dtype=torch.float32, device=dev)
    elif theta0 is not None:
        lab = None
        w, mu, cov = (a.to(device=dev, dtype=torch.float32).contiguous().clone()
                      for a in theta0)
        if w.shape != (k,) or mu.shape != (k, 3) or cov.shape != (k, 3, 3):
            raise ValueError("theta0 shapes must be (K,), (K,3), (K,3,3)")
    else:
        raise ValueError("give labels or theta0")
    L = torch.empty(iters + 1, dtype=torch.float64, device=dev)
    _lib.check(lib.gmm_fit_noalloc(_ptr(pts), n, k, _ptr(lab), _ptr(w), _ptr(mu),
                                   _ptr(cov), _ptr(L), ctypes.byref(opts),
                                   _stream(dev)))
    return FitResult(w, mu, cov, L)


def fit_batched(points_list, ks, iters=100, reg_covar=1e-3, labels_list=None,
                theta0_list=None, moment_mode="shifted", workspace=None):
    """Fit one GMM per frame, all frames in one batched submission.

    points_list: float32 (N_f, 3) CUDA tensors; ks: K_f per frame; start
    from per-frame hard labels or theta0 = (w, mu, cov) per frame.  Returns
    one FitResult per frame (views into concatenated outputs)."""
    import numpy as np
    torch = _torch()
    lib = _lib.load()
    B = len(points_list)
    if B == 0 or len(ks) != B:
        raise ValueError("need one K per frame")
    dev = points_list[0].device
    pts = torch.cat([_check_points(p) for p in points_list]).contiguous()
    pt_off = np.zeros(B + 1, np.int64)
    pt_off[1:] = np.cumsum([p.shape[0] for p in points_list])
    k_off = np.zeros(B + 1, np.int32)
    k_off[1:] = np.cumsum(ks)
    Kt = int(k_off[-1])
    opts = _lib.FitOpts(int(iters), float(reg_covar),
                        {"shifted": 0, "two_pass": 1}[moment_mode], 0)
    if labels_list is not None:
        lab = torch.cat([l.to(device=dev, dtype=torch.int32) for l in labels_list]).contiguous()
        w = torch.empty(Kt, dtype=torch.float32, device=dev)
        mu = torch.empty(Kt, 3, dtype=torch.float32, device=dev)
        cov = torch.empty(Kt, 3, 3, dtype=torch.float32, device=dev)
    elif theta0_list is not None:
        lab = None
        w = torch.cat([t[0].to(device=dev, dtype=torch.float32) for t in theta0_list]).contiguous()
        mu = torch.cat([t[1].to(device=dev, dtype=torch.float32) for t in theta0_list]).contiguous()
        cov = torch.cat([t[2].to(device=dev, dtype=torch.float32) for t in theta0_list]).contiguous()
    else:
        raise ValueError("give labels_list or theta0_list")
    L = torch.empty(B, iters + 1, dtype=torch.float64, device=dev)
    po = pt_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    ko = k_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    need = lib.gmm_fit_batched_workspace_size(B, po, ko, ctypes.byref(opts))
    if need == 0:
        _lib.check(lib.gmm_fit_batched(B, None, po, ko, None, None, None, None,
                                       None, ctypes.byref(opts), None, 0, None))
    ws = workspace if workspace is not None and workspace.numel() >= need \
        else _workspace(need, dev)
    _lib.check(lib.gmm_fit_batched(B, _ptr(pts), po, ko, _ptr(lab), _ptr(w),
                                   _ptr(mu), _ptr(cov), _ptr(L),
                                   ctypes.byref(opts), _ptr(ws), ws.numel(),
                                   _stream(dev)))
    out = []
    for f in range(B):
        a, b = int(k_off[f]), int(k_off[f + 1])
        out.append(FitResult(w[a:b], mu[a:b], cov[a:b], L[f]))
    return out


def fit_batched_workspace_bytes(ns, ks, iters=100):
    import numpy as np
    lib = _lib.load()
    B = len(ns)
    pt_off = np.zeros(B + 1, np.int64)
    pt_off[1:] = np.cumsum(ns)
    k_off = np.zeros(B + 1, np.int32)
    k_off[1:] = np.cumsum(ks)
    opts = _lib.FitOpts(int(iters), 1e-3, 0, 0)
    return int(lib.gmm_fit_batched_workspace_size(
        B, pt_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        k_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(opts)))


def fit_workspace_bytes(n, k, iters=100, reg_covar=1e-3, moment_mode="shifted"):
    lib = _lib.load()
    opts = _lib.FitOpts(int(iters), float(reg_covar),
                        {"shifted": 0, "two_pass": 1}[moment_mode], 0)
    return int(lib.gmm_fit_workspace_size(n, k, ctypes.byref(opts)))


def _gmm_args(w, mu, cov, dev):
    torch = _torch()
    w = w.to(device=dev, dtype=torch.float32).contiguous()
    mu = mu.to(device=dev, dtype=torch.float32).contiguous()
    cov = cov.to(device=dev, dtype=torch.float32).contiguous()
    k = w.shape[0]
    if mu.shape != (k, 3) or cov.shape != (k, 3, 3):
        raise ValueError("mixture shapes must be (K,), (K,3), (K,3,3)")
    return w, mu, cov, k


def _device_status(ws, dev):
    """Waits for the stream and raises GmmError when the kernels flagged a
    device-side condition (non-SPD covariance, weight <= 0, non-finite
    point or result) in the workspace's status word."""
    lib = _lib.load()
    _lib.check(lib.gmm_workspace_status(_ptr(ws), _stream(dev)))


def loglik(points, w, mu, cov, pose6=None, return_lse=False, check=True):
    """L = sum_n ln sum_b w_b N(R x_n + t | mu_b, cov_b) (float64 scalar on
    the device).  pose6 = (omega, t) float32 (6,) or None.

    check=True waits for the result and raises GmmError on a device-side
    error (a covariance that is not SPD, a weight <= 0, a non-finite
    point); check=False returns without waiting (the result is then
    unspecified after such an error)."""
    torch = _torch()
    lib = _lib.load()
    pts = _check_points(points)
    dev = pts.device
    n = pts.shape[0]
    w, mu, cov, k = _gmm_args(w, mu, cov, dev)
    pose = None if pose6 is None else pose6.to(device=dev, dtype=torch.float32).contiguous()
    out = torch.empty((), dtype=torch.float64, device=dev)
    lse = torch.empty(n, dtype=torch.float32, device=dev) if return_lse else None
    need = lib.gmm_loglik_workspace_size(n, k)
    if need == 0:
        _lib.check(lib.gmm_loglik(None, n, None, k, None, None, None, None,
                                  None, None, 0, None))
    ws = _workspace(need, dev)
    _lib.check(lib.gmm_loglik(_ptr(pts), n, _ptr(pose), k, _ptr(w), _ptr(mu),
                              _ptr(cov), _ptr(out), _ptr(lse), _ptr(ws),
                              ws.numel(), _stream(dev)))
    if check:
        _device_status(ws, dev)
    return (out, lse) if return_lse else out


def loglik_backward(points, w, mu, cov, pose6=None, grad_L=None,
                    need=("pose", "pts", "w", "mu", "cov"), check=True):
    """Gradient of grad_L * L with respect to pose (omega, t), points,
    weights, means and covariances; returns a dict of float32 tensors
    (None for keys not in ``need``).  ``check`` as for loglik (a component
    whose covariance is not SPD has NaN gradients)."""
    torch = _torch()
    lib = _lib.load()
    pts = _check_points(points)
    dev = pts.device
    n = pts.shape[0]
    w, mu, cov, k = _gmm_args(w, mu, cov, dev)
    pose = None if pose6 is None else pose6.to(device=dev, dtype=torch.float32).contiguous()
    shapes = dict(pose=(6,), pts=(n, 3), w=(k,), mu=(k, 3), cov=(k, 3, 3))
    g = {key: (torch.empty(shapes[key], dtype=torch.float32, device=dev)
               if key in need else None) for key in shapes}
    if pose is None:
        g["pose"] = None
    gl = None if grad_L is None else grad_L.to(device=dev, dtype=torch.float64).contiguous()
    nb = lib.gmm_loglik_backward_workspace_size(n, k)
    if nb == 0:
        _lib.check(lib.gmm_loglik_backward(None, n, None, k, None, None, None,
                                           None, None, None, None, None, None,
                                           None, 0, None))
    ws = _workspace(nb, dev)
    _lib.check(lib.gmm_loglik_backward(
        _ptr(pts), n, _ptr(pose), k, _ptr(w), _ptr(mu), _ptr(cov), _ptr(gl),
        _ptr(g["pose"]), _ptr(g["pts"]), _ptr(g["w"]), _ptr(g["mu"]),
        _ptr(g["cov"]), _ptr(ws), ws.numel(), _stream(dev)))
    if check:
        _device_status(ws, dev)
    return g


def _make_autograd():
    torch = _torch()

    class GMMLogLik(torch.autograd.Function):
        """L(points, pose6, w, mu, cov) with a hand-written backward kernel."""

        @staticmethod
        def forward(ctx, points, pose6, w, mu, cov):
            out = loglik(points, w, mu, cov, pose6=pose6)
            ctx.save_for_backward(points, pose6, w, mu, cov)
            return out

        @staticmethod
        def backward(ctx, grad_out):
            points, pose6, w, mu, cov = ctx.saved_tensors
            need = []
            for key, i in (("pts", 0), ("pose", 1), ("w", 2), ("mu", 3), ("cov", 4)):
                if ctx.needs_input_grad[i]:
                    need.append(key)
            g = loglik_backward(points, w, mu, cov, pose6=pose6,
                                grad_L=grad_out, need=tuple(need))
            return g["pts"], g["pose"], g["w"], g["mu"], g["cov"]

    return GMMLogLik


class _LazyAutograd:
    _cls = None

    def __getattr__(self, name):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _make_autograd()
        return getattr(_LazyAutograd._cls, name)


GMMLogLik = _LazyAutograd()


def kmeanspp_workspace_bytes(n, k):
    return int(_lib.load().gmm_kmeanspp_workspace_size(int(n), int(k)))


def kmeanspp(points, k, seed=0, u=None, workspace=None):
    """k-means++ seeding on the GPU (gmm_kmeanspp): K centres by D^2
    sampling and the nearest-centre label of every point, the start of a
    fit (``fit(points, k, labels=labels)``).

    ``u`` holds the K draws in [0, 1) (float64, any device); by default
    they come from ``numpy.random.default_rng(seed).random(k)``.  Returns
    (labels int32 (N,), centre indices int64 (K,)), on the points' device."""
    import numpy as np
    torch = _torch()
    lib = _lib.load()
    pts = _check_points(points)
    dev = pts.device
    n, k = pts.shape[0], int(k)
    if u is None:
        u = np.random.default_rng(seed).random(k)
    ut = torch.as_tensor(u, dtype=torch.float64).to(dev).contiguous()
    if ut.shape != (k,):
        raise ValueError("u must hold k draws")
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    centres = torch.empty(k, dtype=torch.int64, device=dev)
    if workspace is None:
        nb = kmeanspp_workspace_bytes(n, k)
        workspace = _workspace(nb, dev) if nb else None
    _lib.check(lib.gmm_kmeanspp(_ptr(pts), n, k, _ptr(ut), _ptr(centres), _ptr(labels),
                                _ptr(workspace),
                                0 if workspace is None else workspace.numel(),
                                _stream(dev)))
    return labels, centres


# ------------------------------------------------------------- 4D model

def fit4_workspace_bytes(n, k, iters=100, reg_covar=1e-3):
    opts = _lib.FitOpts(int(iters), float(reg_covar), 0, 0)
    return int(_lib.load().gmm4_fit_workspace_size(int(n), int(k), ctypes.byref(opts)))


def fit4(points, k, iters=100, reg_covar=1e-3, labels=None, theta0=None,
         moment_mode="shifted", sync=True, workspace=None):
    """EM fit of a K-component 4D mixture to ``points`` (float32 (N, 4) =
    (x, y, z, intensity) on the GPU); start from hard ``labels`` or from
    ``theta0 = (w (K,), mu (K, 4), cov (K, 4, 4))``.  Returns a FitResult
    with means (K, 4) and covariances (K, 4, 4).  With a caller-held
    ``workspace`` (uint8 tensor of at least fit4_workspace_bytes), repeated
    calls replay a captured graph."""
    torch = _torch()
    lib = _lib.load()
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise TypeError("points must be a CUDA (HIP) torch tensor")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 4:
        raise ValueError("points must be float32 of shape (N, 4)")
    pts = points.contiguous()
    dev = pts.device
    n = pts.shape[0]
    opts = _lib.FitOpts(int(iters), float(reg_covar),
                        {"shifted": _lib.GMM_MOMENTS_SHIFTED,
                         "two_pass": _lib.GMM_MOMENTS_TWO_PASS}[moment_mode],
                        0 if sync else _lib.GMM_FLAG_ASYNC)
    if labels is not None:
        lab = labels.to(device=dev, dtype=torch.int32).contiguous()
        if lab.shape != (n,):
            raise ValueError("labels must have shape (N,)")
        w = torch.empty(k, dtype=torch.float32, device=dev)
        mu = torch.empty(k, 4, dtype=torch.float32, device=dev)
        cov = torch.empty(k, 4, 4, dtype=torch.float32, device=dev)
    elif theta0 is not None:
        lab = None
        w, mu, cov = (a.to(device=dev, dtype=torch.float32).contiguous().clone()
                      for a in theta0)
        if w.shape != (k,) or mu.shape != (k, 4) or cov.shape != (k, 4, 4):
            raise ValueError("theta0 shapes must be (K,), (K,4), (K,4,4)")
    else:
        raise ValueError("give labels or theta0")
    L = torch.empty(iters + 1, dtype=torch.float64, device=dev)
    need = lib.gmm4_fit_workspace_size(n, k, ctypes.byref(opts))
    if need == 0:
        _lib.check(lib.gmm4_fit(None, n, k, None, None, None, None, None,
                                ctypes.byref(opts), None, 0, None))
    ws = workspace if workspace is not None and workspace.numel() >= need \
        else _workspace(need, dev)
    _lib.check(lib.gmm4_fit(_ptr(pts), n, k, _ptr(lab), _ptr(w), _ptr(mu), _ptr(cov),
                            _ptr(L), ctypes.byref(opts), _ptr(ws), ws.numel(),
                            _stream(dev)))
    return FitResult(w, mu, cov, L)


def _mixture4(w, mu, cov, dev):
    torch = _torch()
    w = w.to(device=dev, dtype=torch.float32).contiguous()
    k = w.shape[0]
    mu = mu.to(device=dev, dtype=torch.float32).contiguous()
    cov = cov.to(device=dev, dtype=torch.float32).contiguous()
    if mu.shape != (k, 4) or cov.shape != (k, 4, 4):
        raise ValueError("a 4D mixture has w (K,), mu (K, 4), cov (K, 4, 4)")
    return w, mu, cov, k


def color_conditional(locs, w, mu, cov, check=True):
    """Expected intensity and its variance at 3D locations ``locs`` (float32
    (M, 3) on the GPU) under a 4D mixture: (E (M,), V (M,)) float32."""
    torch = _torch()
    lib = _lib.load()
    locs = _check_points(locs)
    dev = locs.device
    m = locs.shape[0]
    w, mu, cov, k = _mixture4(w, mu, cov, dev)
    E = torch.empty(m, dtype=torch.float32, device=dev)
    V = torch.empty(m, dtype=torch.float32, device=dev)
    ws = _workspace(max(lib.gmm4_color_conditional_workspace_size(k), 256), dev)
    _lib.check(lib.gmm4_color_conditional(_ptr(locs), m, k, _ptr(w), _ptr(mu), _ptr(cov),
                                          _ptr(E), _ptr(V), _ptr(ws), ws.numel(),
                                          _stream(dev)))
    if check:
        _device_status(ws, dev)
    return E, V


def joint_dist_sample(w, mu, cov, m, seed=0, u=None, z=None, check=True):
    """m samples (float32 (m, 4)) of a 4D mixture and their components
    (int32 (m,)).  The draws: u (m,) uniforms in [0, 1) choose the component,
    z (m, 4) standard normals the offset (numpy arrays or device tensors); by
    default both come from numpy's default_rng(seed) (u first, then z)."""
    import numpy as np
    torch = _torch()
    lib = _lib.load()
    dev = torch.device("cuda", torch.cuda.current_device()) if not hasattr(w, "device") \
        else w.device
    w, mu, cov, k = _mixture4(w, mu, cov, dev)
    if u is None or z is None:
        rng = np.random.default_rng(seed)
        u = rng.random(m) if u is None else u
        z = rng.standard_normal((m, 4)) if z is None else z
    u = (u.to(dev, torch.float64) if torch.is_tensor(u)
         else torch.as_tensor(np.asarray(u, np.float64)).to(dev)).contiguous()
    z = (z.to(dev, torch.float32) if torch.is_tensor(z)
         else torch.as_tensor(np.asarray(z, np.float32)).to(dev)).contiguous()
    if u.shape != (m,) or z.shape != (m, 4):
        raise ValueError("u must be (m,) and z (m, 4)")
    out = torch.empty(m, 4, dtype=torch.float32, device=dev)
    comp = torch.empty(m, dtype=torch.int32, device=dev)
    ws = _workspace(max(lib.gmm4_joint_dist_sample_workspace_size(k), 256), dev)
    _lib.check(lib.gmm4_joint_dist_sample(k, _ptr(w), _ptr(mu), _ptr(cov), m, _ptr(u),
                                          _ptr(z), _ptr(out), _ptr(comp), _ptr(ws),
                                          ws.numel(), _stream(dev)))
    if check:
        _device_status(ws, dev)
    return out, comp


def meanshift_workspace_bytes(n, d):
    return int(_lib.load().gmm_meanshift_workspace_size(int(n), int(d)))


def meanshift(points, bandwidth, max_iter=300, seeds=False, workspace=None):
    """Number of mixture components for a bandwidth by flat-kernel mean shift
    over binned seeds (gmm_meanshift).  points: float32 (N, 3) or (N, 4) on
    the GPU.  Returns (modes float64 (K, d), weights int64 (K,), info dict);
    the modes are in seed order (lexicographic order of their seeds' bins).
    seeds=True adds the per-seed results to info: seed_modes (S, d),
    seed_weights, seed_iters and seed_status (1 kept, 2 removed by the merge,
    3 dropped), S = info["n_seeds"]."""
    torch = _torch()
    lib = _lib.load()
    if not (hasattr(points, "is_cuda") and points.is_cuda):
        raise ValueError("points must be a CUDA tensor")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] not in (3, 4):
        raise ValueError("points must be float32 (N, 3) or (N, 4)")
    points = points.contiguous()
    dev = points.device
    n, d = points.shape
    cap = max(n, 1)
    modes = torch.empty(cap, d, dtype=torch.float64, device=dev)
    weights = torch.empty(cap, dtype=torch.int64, device=dev)
    sm = sw = si = ss = None
    if seeds:
        sm = torch.empty(cap, d, dtype=torch.float64, device=dev)
        sw, si, ss = (torch.empty(cap, dtype=torch.int32, device=dev) for _ in range(3))
    if workspace is None:
        workspace = _workspace(max(lib.gmm_meanshift_workspace_size(n, d), 256), dev)
    info = _lib.MeanShiftInfo()
    _lib.check(lib.gmm_meanshift(
        _ptr(points) if n else None, n, d, float(bandwidth), int(max_iter), _ptr(modes),
        _ptr(weights), cap, _ptr(sm) if seeds else None, _ptr(sw) if seeds else None,
        _ptr(si) if seeds else None, _ptr(ss) if seeds else None, ctypes.byref(info),
        _ptr(workspace), workspace.numel(), _stream(dev)))
    K = int(info.n_modes)
    out = {"n_seeds": int(info.n_seeds), "n_modes": K, "rounds": int(info.rounds),
           "max_iters": int(info.max_iters)}
    if seeds:
        S = out["n_seeds"]
        out.update(seed_modes=sm[:S], seed_weights=sw[:S], seed_iters=si[:S],
                   seed_status=ss[:S])
    return modes[:K], weights[:K], out


def _mixture3(mix, dev):
    torch = _torch()
    w, mu, cov = (torch.as_tensor(a).to(dev, torch.float32).contiguous() for a in mix)
    k = w.shape[0]
    if w.shape != (k,) or mu.shape != (k, 3) or cov.shape != (k, 3, 3):
        raise ValueError("a mixture is (w (K,), mu (K, 3), cov (K, 3, 3))")
    return w, mu, cov, k


def d2d_objective(pose6, src, tgt, variant="anisotropic", check=True):
    """f = ln sum_ij pi_i tau_j N(R mu_i + t; nu_j, R Sigma_i R^T + Lambda_j)
    and df/d(omega, t) at pose6 = (omega, t) (gmm_d2d_objective).  src, tgt:
    (w, mu, cov) mixtures; variant "anisotropic" or "isoplanar".  Returns
    (f float, grad float64 numpy (6,))."""
    torch = _torch()
    lib = _lib.load()
    dev = torch.device("cuda", torch.cuda.current_device())
    if hasattr(src[0], "device") and src[0].device.type == "cuda":
        dev = src[0].device
    w, mu, cov, m = _mixture3(src, dev)
    tw, tmu, tcov, n = _mixture3(tgt, dev)
    var = {"anisotropic": _lib.GMM_D2D_ANISOTROPIC, "isoplanar": _lib.GMM_D2D_ISOPLANAR}[variant]
    p = torch.as_tensor(pose6, dtype=torch.float64).reshape(6).to(dev)
    out = torch.empty(7, dtype=torch.float64, device=dev)
    ws = _workspace(max(lib.gmm_d2d_workspace_size(m, n), 256), dev)
    _lib.check(lib.gmm_d2d_objective(_ptr(p), m, _ptr(w), _ptr(mu), _ptr(cov), n, _ptr(tw),
                                     _ptr(tmu), _ptr(tcov), var, _ptr(out), _ptr(ws),
                                     ws.numel(), _stream(dev)))
    if check:
        _device_status(ws, dev)
    o = out.cpu().numpy()
    return float(o[0]), o[1:]


def d2d_register(src, tgt, T0=None, iters_iso=30, iters_aniso=30, check=True):
    """Isoplanar then anisotropic D2D registration of the mixture src to tgt
    from the 4 x 4 transform T0 (identity by default), gmm_d2d_register.
    Returns (T float64 (4, 4) tensor on the device, history float64 tensor
    (f per stage start and accepted iteration, NaN after the last), counts
    int32 tensor (2,))."""
    import numpy as np
    torch = _torch()
    lib = _lib.load()
    dev = torch.device("cuda", torch.cuda.current_device())
    if hasattr(src[0], "device") and src[0].device.type == "cuda":
        dev = src[0].device
    w, mu, cov, m = _mixture3(src, dev)
    tw, tmu, tcov, n = _mixture3(tgt, dev)
    T0 = np.eye(4) if T0 is None else T0
    T0 = torch.as_tensor(T0, dtype=torch.float64).reshape(4, 4).to(dev).contiguous()
    T = torch.empty(4, 4, dtype=torch.float64, device=dev)
    hist = torch.empty(iters_iso + iters_aniso + 2, dtype=torch.float64, device=dev)
    counts = torch.empty(2, dtype=torch.int32, device=dev)
    ws = _workspace(max(lib.gmm_d2d_workspace_size(m, n), 256), dev)
    _lib.check(lib.gmm_d2d_register(_ptr(T0), m, _ptr(w), _ptr(mu), _ptr(cov), n, _ptr(tw),
                                    _ptr(tmu), _ptr(tcov), int(iters_iso), int(iters_aniso),
                                    _ptr(T), _ptr(hist), _ptr(counts), _ptr(ws), ws.numel(),
                                    _stream(dev)))
    if check:
        _device_status(ws, dev)
    return T, hist, counts
