"""ctypes binding of libgmm.so (the C ABI declared in include/gmm.h).

Only argument marshalling lives here: every step of the fit and of the
log-likelihood runs in the HIP library.  Loading fails loudly when the
library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgmm.so")

GMM_OK = 0
GMM_ERR_INVALID_ARG = 1
GMM_ERR_NOT_SPD = 2
GMM_ERR_NONFINITE = 3
GMM_ERR_OOM = 4
GMM_ERR_DEVICE = 5
GMM_ERR_UNSUPPORTED = 6
GMM_MOMENTS_SHIFTED = 0
GMM_MOMENTS_TWO_PASS = 1
GMM_FLAG_ASYNC = 1
GMM_FLAG_DETERMINISTIC = 2
GMM_MAX_K = 1024
GMM_FIT_NOALLOC_MAX_BYTES = 64 << 20
GMM_D2D_ANISOTROPIC = 0
GMM_D2D_ISOPLANAR = 1

EXPORTS = (
    "gmm_status_string", "gmm_last_error", "gmm_workspace_status",
    "gmm_fit_workspace_size", "gmm_fit", "gmm_fit_noalloc",
    "gmm_loglik_workspace_size", "gmm_loglik",
    "gmm_loglik_backward_workspace_size", "gmm_loglik_backward",
    "gmm_fit_batched_workspace_size", "gmm_fit_batched", "gmm_fit_batched_config",
    "gmm_set_autotune", "gmm_tile_config",
    "gmm_profile_enable", "gmm_profile_read", "gmm_profile_pairs",
    "gmm_kmeanspp_workspace_size", "gmm_kmeanspp",
    "gmm4_fit_workspace_size", "gmm4_fit",
    "gmm4_color_conditional_workspace_size", "gmm4_color_conditional",
    "gmm4_joint_dist_sample_workspace_size", "gmm4_joint_dist_sample",
    "gmm_meanshift_workspace_size", "gmm_meanshift",
    "gmm_d2d_workspace_size", "gmm_d2d_objective", "gmm_d2d_register",
)


class GmmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("gmm status %d: %s" % (status, msg))
        self.status = status


class MeanShiftInfo(ctypes.Structure):
    _fields_ = [("n_seeds", ctypes.c_int64), ("n_modes", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("max_iters", ctypes.c_int32)]


class FitOpts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("reg_covar", ctypes.c_double),
                ("moment_mode", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("tol", ctypes.c_double)]


_lib = None


def load():
    """Load libgmm.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libgmm.so is not built (%s); run `python -m "
            "paper_2307_00071_amd.build` or __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    lib.gmm_status_string.argtypes = [ctypes.c_int]
    lib.gmm_status_string.restype = ctypes.c_char_p
    lib.gmm_last_error.argtypes = []
    lib.gmm_last_error.restype = ctypes.c_char_p
    lib.gmm_workspace_status.argtypes = [vp, vp]
    lib.gmm_workspace_status.restype = ctypes.c_int
    lib.gmm_fit_workspace_size.argtypes = [i64, i32, ctypes.POINTER(FitOpts)]
    lib.gmm_fit_workspace_size.restype = sz
    lib.gmm_fit.argtypes = [vp, i64, i32, vp, vp, vp, vp, vp,
                            ctypes.POINTER(FitOpts), vp, sz, vp]
    lib.gmm_fit.restype = ctypes.c_int
    lib.gmm_fit_noalloc.argtypes = [vp, i64, i32, vp, vp, vp, vp, vp,
                                    ctypes.POINTER(FitOpts), vp]
    lib.gmm_fit_noalloc.restype = ctypes.c_int
    lib.gmm_loglik_workspace_size.argtypes = [i64, i32]
    lib.gmm_loglik_workspace_size.restype = sz
    lib.gmm_loglik.argtypes = [vp, i64, vp, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.gmm_loglik.restype = ctypes.c_int
    lib.gmm_loglik_backward_workspace_size.argtypes = [i64, i32]
    lib.gmm_loglik_backward_workspace_size.restype = sz
    lib.gmm_loglik_backward.argtypes = [vp, i64, vp, i32, vp, vp, vp, vp, vp,
                                        vp, vp, vp, vp, vp, sz, vp]
    lib.gmm_loglik_backward.restype = ctypes.c_int
    lib.gmm_fit_batched_workspace_size.argtypes = [
        i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
        ctypes.POINTER(FitOpts)]
    lib.gmm_fit_batched_workspace_size.restype = sz
    lib.gmm_fit_batched.argtypes = [
        i32, vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
        vp, vp, vp, vp, vp, ctypes.POINTER(FitOpts), vp, sz, vp]
    lib.gmm_fit_batched.restype = ctypes.c_int
    lib.gmm_fit_batched_config.argtypes = [
        i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
    lib.gmm_fit_batched_config.restype = ctypes.c_char_p
    lib.gmm_set_autotune.argtypes = [ctypes.c_int]
    lib.gmm_set_autotune.restype = ctypes.c_int
    lib.gmm_tile_config.argtypes = [i64, i32]
    lib.gmm_tile_config.restype = ctypes.c_char_p
    lib.gmm_profile_enable.argtypes = [ctypes.c_int]
    lib.gmm_profile_enable.restype = ctypes.c_int
    lib.gmm_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.gmm_profile_read.restype = ctypes.c_int
    lib.gmm_profile_pairs.argtypes = [ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.gmm_profile_pairs.restype = ctypes.c_int
    lib.gmm_kmeanspp_workspace_size.argtypes = [i64, i32]
    lib.gmm_kmeanspp_workspace_size.restype = sz
    lib.gmm_kmeanspp.argtypes = [vp, i64, i32, vp, vp, vp, vp, sz, vp]
    lib.gmm_kmeanspp.restype = ctypes.c_int
    lib.gmm4_fit_workspace_size.argtypes = [i64, i32, ctypes.POINTER(FitOpts)]
    lib.gmm4_fit_workspace_size.restype = sz
    lib.gmm4_fit.argtypes = [vp, i64, i32, vp, vp, vp, vp, vp,
                             ctypes.POINTER(FitOpts), vp, sz, vp]
    lib.gmm4_fit.restype = ctypes.c_int
    lib.gmm4_color_conditional_workspace_size.argtypes = [i32]
    lib.gmm4_color_conditional_workspace_size.restype = sz
    lib.gmm4_color_conditional.argtypes = [vp, i64, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.gmm4_color_conditional.restype = ctypes.c_int
    lib.gmm4_joint_dist_sample_workspace_size.argtypes = [i32]
    lib.gmm4_joint_dist_sample_workspace_size.restype = sz
    lib.gmm4_joint_dist_sample.argtypes = [i32, vp, vp, vp, i64, vp, vp, vp, vp, vp, sz, vp]
    lib.gmm4_joint_dist_sample.restype = ctypes.c_int
    lib.gmm_meanshift_workspace_size.argtypes = [i64, i32]
    lib.gmm_meanshift_workspace_size.restype = sz
    lib.gmm_meanshift.argtypes = [vp, i64, i32, ctypes.c_double, i32, vp, vp, i64,
                                  vp, vp, vp, vp, ctypes.POINTER(MeanShiftInfo), vp, sz, vp]
    lib.gmm_meanshift.restype = ctypes.c_int
    lib.gmm_d2d_workspace_size.argtypes = [i32, i32]
    lib.gmm_d2d_workspace_size.restype = sz
    lib.gmm_d2d_objective.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp, vp, i32, vp, vp, sz, vp]
    lib.gmm_d2d_objective.restype = ctypes.c_int
    lib.gmm_d2d_register.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp, vp, i32, i32, vp, vp,
                                     vp, vp, sz, vp]
    lib.gmm_d2d_register.restype = ctypes.c_int
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != GMM_OK:
        lib = load()
        detail = lib.gmm_last_error().decode() or lib.gmm_status_string(status).decode()
        raise GmmError(status, detail)


def profile_enable(reps: int) -> None:
    """reps >= 1: time each E+M tile pass of gmm_fit over reps back-to-back
    launches between one event pair; 0: off."""
    check(load().gmm_profile_enable(int(reps)))


def profile_read():
    """(summed E+M tile-kernel time in ms, launch count) since the last read."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    check(load().gmm_profile_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def profile_pairs():
    """(evaluated, all) (tile, component) pairs of the timed E+M launches
    since the last call."""
    ev = ctypes.c_int64(0)
    al = ctypes.c_int64(0)
    check(load().gmm_profile_pairs(ctypes.byref(ev), ctypes.byref(al)))
    return ev.value, al.value


def set_autotune(on: bool) -> None:
    check(load().gmm_set_autotune(1 if on else 0))


def tile_config(n: int, k: int) -> str:
    """Name of the tile shape a fit of n points, k components uses now."""
    return load().gmm_tile_config(int(n), int(k)).decode()


def batch_config(ns, ks) -> str:
    """Soft-pass shape of a batched fit of frames with ns points and ks
    components ("" when autotuning will pick it at the call)."""
    import numpy as np
    B = len(ns)
    pt_off = np.zeros(B + 1, np.int64)
    pt_off[1:] = np.cumsum(ns)
    k_off = np.zeros(B + 1, np.int32)
    k_off[1:] = np.cumsum(ks)
    return load().gmm_fit_batched_config(
        B, pt_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        k_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))).decode()
