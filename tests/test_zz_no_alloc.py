"""gmm_fit_noalloc (the fit for callers that cannot allocate) against
gmm_fit through the C ABI: the same kernels on the same workspace layout,
so the outputs agree bit for bit; checked on two calls in a row, the second
with a smaller input (the shared per-GPU array keeps the first call's
contents), and against the FP64 oracle's log-likelihood bar."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2307_00071_amd import _lib, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _case(name):
    print("case:", name, flush=True)


def _subset(n, seed):
    X = synth.depth_frame(seed)
    rng = np.random.default_rng(seed + 3)
    return np.ascontiguousarray(X[np.sort(rng.choice(X.shape[0], n, replace=False))])


def _call(entry, X, K, T, lab, mode=0):
    """Runs gmm_fit (entry == "fit", caller workspace) or gmm_fit_noalloc
    through ctypes; returns (status, w, mu, cov, L) as numpy arrays."""
    lib = _lib.load()
    n = X.shape[0]
    pts = torch.from_numpy(X).to(DEV)
    labt = torch.from_numpy(lab.astype(np.int32)).to(DEV)
    w = torch.full((K,), np.nan, dtype=torch.float32, device=DEV)
    mu = torch.full((K, 3), np.nan, dtype=torch.float32, device=DEV)
    cov = torch.full((K, 3, 3), np.nan, dtype=torch.float32, device=DEV)
    L = torch.full((T + 1,), np.nan, dtype=torch.float64, device=DEV)
    opts = _lib.FitOpts(T, 1e-3, mode, 0)
    stream = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    if entry == "fit":
        need = lib.gmm_fit_workspace_size(n, K, ctypes.byref(opts))
        ws = torch.empty(need, dtype=torch.uint8, device=DEV)
        st = lib.gmm_fit(p(pts), n, K, p(labt), p(w), p(mu), p(cov), p(L),
                         ctypes.byref(opts), p(ws), need, stream)
    else:
        st = lib.gmm_fit_noalloc(p(pts), n, K, p(labt), p(w), p(mu), p(cov), p(L),
                                 ctypes.byref(opts), stream)
    torch.cuda.synchronize()
    return (st,) + tuple(t.cpu().numpy() for t in (w, mu, cov, L))


@pytest.mark.parametrize("mode", [0, 1])
def test_noalloc_matches_fit_on_two_calls(mode):
    lib = _lib.load()
    for n, K, T, seed in ((150000, 100, 12, 0), (20011, 37, 8, 1)):
        _case("noalloc mode=%d n=%d K=%d T=%d" % (mode, n, K, T))
        X = _subset(n, seed)
        lab = synth.kmeanspp_labels(X, K, seed + 1)
        opts = _lib.FitOpts(T, 1e-3, mode, 0)
        assert lib.gmm_fit_workspace_size(n, K, ctypes.byref(opts)) <= \
            _lib.GMM_FIT_NOALLOC_MAX_BYTES
        ref = _call("fit", X, K, T, lab, mode)
        got = _call("noalloc", X, K, T, lab, mode)
        assert ref[0] == 0 and got[0] == 0, (ref[0], got[0])
        for a, b in zip(got[1:], ref[1:]):
            np.testing.assert_array_equal(a, b)
        Lr = oracle.fit(X, K, 1e-3, T, labels=lab)[3]
        err = np.abs(got[4] - Lr) / np.maximum(np.abs(Lr), n)
        assert err.max() <= 1e-4, err.max()


def test_noalloc_rejects_what_it_cannot_hold():
    """A fit larger than the scratch array, and the asynchronous flag, are
    refused on the host before anything is enqueued; a good call after
    them still works."""
    _case("noalloc limits")
    lib = _lib.load()
    n, K = 2_000_000, 1000
    opts = _lib.FitOpts(2, 1e-3, 0, 0)
    assert lib.gmm_fit_workspace_size(n, K, ctypes.byref(opts)) > \
        _lib.GMM_FIT_NOALLOC_MAX_BYTES
    dummy = torch.zeros(16, dtype=torch.float32, device=DEV)
    p = ctypes.c_void_p(dummy.data_ptr())
    st = lib.gmm_fit_noalloc(p, n, K, None, p, p, p, None, ctypes.byref(opts), None)
    assert st == 6, st                               # GMM_ERR_UNSUPPORTED
    assert b"scratch" in lib.gmm_last_error()
    aopts = _lib.FitOpts(2, 1e-3, 0, _lib.GMM_FLAG_ASYNC)
    st = lib.gmm_fit_noalloc(p, 100, 2, None, p, p, p, None, ctypes.byref(aopts), None)
    assert st == 1, st                               # GMM_ERR_INVALID_ARG
    X = _subset(5000, 4)
    lab = synth.kmeanspp_labels(X, 8, 2)
    ref = _call("fit", X, 8, 3, lab)
    got = _call("noalloc", X, 8, 3, lab)
    assert got[0] == 0
    for a, b in zip(got[1:], ref[1:]):
        np.testing.assert_array_equal(a, b)
