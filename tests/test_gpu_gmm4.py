"""GPU parity of the 4D (x, y, z, intensity) mixture calls (gmm4_fit,
gmm4_color_conditional, gmm4_joint_dist_sample, through the C ABI) against
the FP64 oracle (oracle/gmm4.py).

Bars:
  * fit, one E+M step from identical float32 parameters: 1e-5 per
    parameter array (Frobenius) and per component with pi_b >= 1e-3
    (tests/parity.py), 1e-5 for L(theta) (floor N); a fixed-iteration fit:
    L(theta_T) within 1e-4 (floor N) at every iteration;
  * conditional intensity, per location: |dE| <= 1e-5 (1 + |E|) and
    |dV| <= 1e-4 V + 1e-7: the FP32 per-component terms carry relative
    errors of a few 1e-7 times the log-term's magnitude (up to ~10 for the
    weights), and V is a difference of two sums of size E^2 taken in FP64;
  * joint sampling: the component of every sample identical (both sides
    walk the same FP64 running sum of the float32 weights), the samples
    within 2 float32 ulps of the oracle's FP64 values.
"""
import numpy as np
import pytest
import torch

from oracle import gmm4 as o4
import paper_2307_00071_amd as gmm
from paper_2307_00071_amd import _lib, synth
from tests.parity import mixture_errors

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _case(name):
    print("case:", name, flush=True)


def _to(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to(DEV, dtype)


def _frame4(n=None, seed=0):
    X = synth.depth_intensity_frame(seed)
    if n is not None:
        rng = np.random.default_rng(seed + 31)
        X = np.ascontiguousarray(X[np.sort(rng.choice(X.shape[0], n, replace=False))])
    return X


def _labels(X, K, seed):
    return synth.kmeanspp_labels(np.ascontiguousarray(X[:, :3]), K, seed)


def _gpu_fit(X, K, T, labels=None, theta0=None, mode="shifted", reg=1e-3):
    r = gmm.fit4(_to(X), K, iters=T, reg_covar=reg,
                 labels=None if labels is None else _to(labels, torch.int32),
                 theta0=None if theta0 is None else tuple(_to(a) for a in theta0),
                 moment_mode=mode)
    torch.cuda.synchronize()
    return tuple(t.cpu().numpy().astype(np.float64) for t in r)


def _theta32(theta):
    return tuple(np.asarray(a, np.float32).astype(np.float64) for a in theta)


@pytest.mark.parametrize("K,n", [(8, 10000), (64, 30011), (1, 999), (300, 20000)])
def test_label_mstep_parity(K, n):
    _case("4D label mstep K=%d n=%d" % (K, n))
    X = _frame4(n, seed=K)
    lab = _labels(X, K, 1)
    w, mu, cov, L = _gpu_fit(X, K, 0, labels=lab)
    ref = o4.mstep_labels(X.astype(np.float64), lab, K, 1e-3)
    e = mixture_errors((w, mu, cov), ref, X)
    print(e, flush=True)
    assert max(e.values()) <= 1e-5, e
    Lr = o4.estep(X, *ref)[0]
    assert abs(L[0] - Lr) <= 1e-5 * max(abs(Lr), n)


@pytest.mark.parametrize("K,n,mode", [(50, 30011, "shifted"), (50, 30011, "two_pass"),
                                      (16, 4099, "shifted"), (200, 25000, "shifted"),
                                      (512, 9000, "shifted")])
def test_one_step_parity(K, n, mode):
    _case("4D one step K=%d n=%d %s" % (K, n, mode))
    X = _frame4(n, seed=K + 1)
    lab = _labels(X, K, 2)
    theta = _theta32(o4.fit(X, K, 1e-3, 2, labels=lab)[:3])
    w, mu, cov, L = _gpu_fit(X, K, 1, theta0=theta, mode=mode)
    wr, mur, covr, L0 = o4.em_step(X.astype(np.float64), *theta, 1e-3)
    e = mixture_errors((w, mu, cov), (wr, mur, covr), X)
    e["L0"] = abs(L[0] - L0) / max(abs(L0), n)
    print(e, flush=True)
    assert max(e.values()) <= 1e-5, e


def test_full_frame_one_step_and_fit():
    """The 640 x 480 depth-intensity frame, K = 100: one step from the same
    theta, then 10 iterations from k-means++ labels (L at every
    iteration)."""
    _case("4D full frame N=307200 K=100")
    X = _frame4()
    N, K = X.shape[0], 100
    lab = _labels(X, K, 1)
    theta = _theta32(o4.fit(X[::7], K, 1e-3, 2, labels=lab[::7])[:3])
    w, mu, cov, L = _gpu_fit(X, K, 1, theta0=theta)
    wr, mur, covr, L0 = o4.em_step(X.astype(np.float64), *theta, 1e-3)
    e = mixture_errors((w, mu, cov), (wr, mur, covr), X)
    e["L0"] = abs(L[0] - L0) / max(abs(L0), N)
    print("one step", e, flush=True)
    assert max(e.values()) <= 1e-5, e
    T = 10
    *_, Lg = _gpu_fit(X, K, T, labels=lab)
    Lr = o4.fit(X, K, 1e-3, T, labels=lab)[3]
    err = np.abs(Lg - Lr) / np.maximum(np.abs(Lr), N)
    print("fit L err", err.max(), flush=True)
    assert err.max() <= 1e-4


def test_fit_final_loglik_and_monotone():
    _case("4D fit T=30")
    X = _frame4(40000, seed=5)
    K, T = 40, 30
    lab = _labels(X, K, 3)
    *_, L = _gpu_fit(X, K, T, labels=lab)
    Lr = o4.fit(X, K, 1e-3, T, labels=lab)[3]
    err = np.abs(L - Lr) / np.maximum(np.abs(Lr), X.shape[0])
    assert err.max() <= 1e-4, err.max()
    *_, L0 = _gpu_fit(X, K, T, labels=lab, reg=0.0)
    assert np.all(np.diff(L0) >= -1e-6 * abs(L0[-1]))


@pytest.mark.parametrize("n,K", [(1, 1), (63, 3), (65, 5), (129, 7)])
def test_small_and_ragged(n, K):
    _case("4D ragged n=%d K=%d" % (n, K))
    X = (np.random.default_rng(n).normal(size=(n, 4)) + 2.0).astype(np.float32)
    lab = (np.arange(n) % K).astype(np.int32)
    w, mu, cov, L = _gpu_fit(X, K, 3, labels=lab)
    wr, mur, covr, Lr = o4.fit(X, K, 1e-3, 3, labels=lab)
    assert np.abs(L - Lr).max() / max(np.abs(Lr).max(), n) <= 1e-5
    e = mixture_errors((w, mu, cov), (wr, mur, covr), X)
    assert max(e["w"], e["mu"], e["cov"]) <= 1e-5, e


def test_empty_component_and_errors():
    _case("4D empty component, errors")
    X = _frame4(8000, seed=9) + np.float32(20.0)
    lab = _labels(X, 6, 1)                       # values 0..5, K = 7: 6 unused
    w, mu, cov, L = _gpu_fit(X, 7, 2, labels=lab)
    wr, mur, covr, Lr = o4.fit(X, 7, 1e-3, 2, labels=lab)
    assert np.all(mu[6] == 0.0)
    np.testing.assert_array_equal(cov[6], np.float32(1e-3) * np.eye(4))
    assert abs(w[6] - wr[6]) <= 1e-5 * wr[6]
    e = mixture_errors((w, mu, cov), (wr, mur, covr), X)
    assert max(e.values()) <= 1e-5, e
    bad = X.copy()
    bad[100, 3] = np.nan
    with pytest.raises(_lib.GmmError) as ei:
        _gpu_fit(bad, 6, 1, labels=lab)
    assert ei.value.status == 3
    with pytest.raises(_lib.GmmError) as ei:
        _gpu_fit(X, 5, 1, labels=lab)            # label 5 out of range for K = 5
    assert ei.value.status == 1
    th = (np.full(2, 0.5), np.zeros((2, 4)), np.stack([np.eye(4), -np.eye(4)]))
    with pytest.raises(_lib.GmmError) as ei:
        _gpu_fit(X, 2, 1, theta0=th)
    assert ei.value.status == 2


# ------------------------------------------------------ conditional intensity

def _fitted4(K=60, n=60000, seed=2):
    X = _frame4(n, seed=seed)
    lab = _labels(X, K, 1)
    th = o4.fit(X, K, 1e-3, 4, labels=lab)[:3]
    return X, tuple(np.asarray(a, np.float32) for a in th)


def _cond_check(locs, th):
    E, V = gmm.color_conditional(_to(locs), *(_to(a) for a in th))
    torch.cuda.synchronize()
    E, V = E.cpu().numpy().astype(np.float64), V.cpu().numpy().astype(np.float64)
    Er, Vr, _ = o4.color_conditional(locs.astype(np.float64), *(a.astype(np.float64) for a in th))
    eE = float((np.abs(E - Er) / (1e-5 * (1 + np.abs(Er)))).max())
    eV = float((np.abs(V - Vr) / (1e-4 * Vr + 1e-7)).max())
    print("conditional: max |dE| / bar %.3g, max |dV| / bar %.3g" % (eE, eV), flush=True)
    assert eE <= 1.0 and eV <= 1.0, (eE, eV)
    return E, V


def test_conditional_at_the_frame_points_and_ragged_sizes():
    _case("4D conditional")
    X, th = _fitted4()
    _cond_check(np.ascontiguousarray(X[:, :3]), th)
    for m in (1, 255, 257, 1001):
        _cond_check(np.ascontiguousarray(X[:m, :3]), th)


def test_conditional_far_locations_and_one_component():
    """Locations 40 m from every component take the exact max-shifted path;
    one component without cross-covariance gives E = mu^i, V = Sigma^ii."""
    _case("4D conditional far / K=1")
    X, th = _fitted4(K=20, n=20000, seed=4)
    locs = np.ascontiguousarray(X[:500, :3] + np.float32(40.0))
    _cond_check(locs, th)
    mu = np.array([[1.0, 2.0, 3.0, 0.4]], np.float32)
    cov = np.diag([0.5, 0.3, 0.2, 0.01]).astype(np.float32)[None]
    E, V = _cond_check(np.ascontiguousarray(X[:300, :3]), (np.ones(1, np.float32), mu, cov))
    np.testing.assert_allclose(E, 0.4, rtol=1e-6)
    np.testing.assert_allclose(V, 0.01, rtol=1e-5)


def test_conditional_device_errors():
    _case("4D conditional errors")
    X, (w, mu, cov) = _fitted4(K=10, n=5000, seed=6)
    locs = np.ascontiguousarray(X[:100, :3])
    bad = cov.copy()
    bad[2] = -np.eye(4)
    with pytest.raises(_lib.GmmError) as ei:
        gmm.color_conditional(_to(locs), _to(w), _to(mu), _to(bad))
    assert ei.value.status == 2
    w0 = w.copy()
    w0[3] = 0.0
    with pytest.raises(_lib.GmmError) as ei:
        gmm.color_conditional(_to(locs), _to(w0), _to(mu), _to(cov))
    assert ei.value.status == 1


# ------------------------------------------------------------ joint sampling

def test_joint_sample_matches_oracle():
    _case("4D joint sample")
    _, th = _fitted4(K=80, n=40000, seed=7)
    for m, seed in ((307200, 1), (1, 2), (1000, 3)):
        rng = np.random.default_rng(seed)
        u = rng.random(m)
        z = rng.standard_normal((m, 4)).astype(np.float32)
        if m > 2:
            u[0], u[1] = 0.0, 1.0 - 2.0 ** -53
        out, comp = gmm.joint_dist_sample(*(_to(a) for a in th), m, u=u, z=z)
        torch.cuda.synchronize()
        ro, rc = o4.joint_sample(*(a.astype(np.float64) for a in th), u, z.astype(np.float64))
        np.testing.assert_array_equal(comp.cpu().numpy(), rc)
        got = out.cpu().numpy()
        ulp = np.spacing(np.abs(ro).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(got - ro) <= 2 * ulp + 1e-30), np.abs(got - ro).max()


def test_joint_sample_statistics_and_errors():
    """Many samples reproduce the mixture's weights and moments (5 standard
    errors); a draw outside [0, 1) and a covariance that is not SPD are
    device errors."""
    _case("4D sample statistics")
    rng = np.random.default_rng(13)
    K = 3
    w = np.array([0.2, 0.5, 0.3], np.float32)
    mu = rng.uniform(-3, 3, (K, 4)).astype(np.float32)
    cov = np.stack([np.diag(rng.uniform(0.1, 1.0, 4)) for _ in range(K)]).astype(np.float32)
    M = 1_000_000
    out, comp = gmm.joint_dist_sample(_to(w), _to(mu), _to(cov), M, seed=5)
    out, comp = out.cpu().numpy().astype(np.float64), comp.cpu().numpy()
    freq = np.bincount(comp, minlength=K) / M
    assert np.all(np.abs(freq - w) <= 5 * np.sqrt(w * (1 - w) / M))
    for b in range(K):
        Y = out[comp == b]
        se = np.sqrt(np.diag(cov[b]) / Y.shape[0])
        assert np.all(np.abs(Y.mean(axis=0) - mu[b]) <= 5 * se)
    with pytest.raises(_lib.GmmError) as ei:
        gmm.joint_dist_sample(_to(w), _to(mu), _to(cov), 4, u=np.array([0.1, 0.2, 1.5, 0.3]),
                              z=np.zeros((4, 4)))
    assert ei.value.status == 1
    bad = cov.copy()
    bad[1, 2, 2] = -1.0
    with pytest.raises(_lib.GmmError) as ei:
        gmm.joint_dist_sample(_to(w), _to(mu), _to(bad), 10, seed=1)
    assert ei.value.status == 2


def test_graph_replay_is_bitwise_equal_to_direct_launches():
    """The same C-ABI call three times with the same buffers: the first runs
    its kernels directly, the second captures them into a graph, the third
    replays it; all three give the same bits, and L agrees with the
    oracle's at the fit bar."""
    import ctypes
    _case("graph replay")
    X = _frame4(20000, seed=4)
    K, T = 40, 12
    lab = _labels(X, K, 2)
    lib = _lib.load()
    pts = _to(X)
    lt = _to(lab, torch.int32)
    w = torch.empty(K, device=DEV)
    mu = torch.empty(K, 4, device=DEV)
    cov = torch.empty(K, 4, 4, device=DEV)
    L = torch.empty(T + 1, dtype=torch.float64, device=DEV)
    opts = _lib.FitOpts(T, 1e-3, 0, 0)
    ws = torch.empty(lib.gmm4_fit_workspace_size(X.shape[0], K, ctypes.byref(opts)),
                     dtype=torch.uint8, device=DEV)
    stream = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    outs = []
    for _ in range(3):
        _lib.check(lib.gmm4_fit(p(pts), X.shape[0], K, p(lt), p(w), p(mu), p(cov), p(L),
                                ctypes.byref(opts), p(ws), ws.numel(), stream))
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy().copy() for t in (w, mu, cov, L)])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            np.testing.assert_array_equal(a, b)
    Lr = o4.fit(X.astype(np.float64), K, 1e-3, T, labels=lab)[3]
    assert np.abs(outs[0][3] - Lr).max() <= 1e-4 * max(np.abs(Lr).max(), X.shape[0])


# ------------------------------------------------------------ culled passes

def _blob4(n, seed):
    """One anisotropic 4D blob: every component of a fit overlaps every tile."""
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(4, 4)) * 0.3
    return (rng.normal(size=(n, 4)) @ A + np.array([2.0, -1.0, 4.0, 0.5])).astype(np.float32)


@pytest.mark.parametrize("what,K,n", [("frame", 7, 5003), ("frame", 100, 40000),
                                      ("frame", 300, 30011), ("blob", 300, 20000)])
def test_culled_passes_equal_dense_passes(what, K, n, monkeypatch):
    """The default culled soft passes (points in Morton order, pairs with a
    zero FP32 weight on the whole tile skipped) against the dense kernel
    (GMM_CULL4=0) on the same fit: L at every iteration within 1e-6 (floor
    N) and the parameters within 1e-5, i.e. equal up to the order of FP32
    additions.  The blob makes every tile see every component, so a tile's
    active components exceed the 128 E rows and the later rows are
    recomputed."""
    _case("4D culled vs dense %s K=%d n=%d" % (what, K, n))
    X = _frame4(n, seed=K + 5) if what == "frame" else _blob4(n, K)
    lab = _labels(X, K, 4)
    T = 5
    wc, muc, covc, Lc = _gpu_fit(X, K, T, labels=lab)
    monkeypatch.setenv("GMM_CULL4", "0")
    wd, mud, covd, Ld = _gpu_fit(X, K, T, labels=lab)
    eL = float(np.max(np.abs(Lc - Ld) / np.maximum(np.abs(Ld), n)))
    e = mixture_errors((wc, muc, covc), (wd, mud, covd), X)
    print("L", eL, e, flush=True)
    assert eL <= 1e-6, eL
    assert max(e.values()) <= 1e-5, e


def test_culled_one_step_with_far_points():
    """One E+M step from fitted parameters on a cloud with 37 points 60 m
    away from every component: those points take the far-point path (their
    own maximum over all K components) in the culled pass; against the
    oracle's step at the one-step bar."""
    _case("4D culled far points")
    X0 = _frame4(20000, seed=12)
    K = 50
    lab = _labels(X0, K, 2)
    theta = _theta32(o4.fit(X0, K, 1e-3, 2, labels=lab)[:3])
    far = (np.random.default_rng(5).normal(size=(37, 4)) * 0.5 +
           np.array([60.0, 60.0, 60.0, 0.5])).astype(np.float32)
    X = np.concatenate([X0[:9000], far, X0[9000:]])
    w, mu, cov, L = _gpu_fit(X, K, 1, theta0=theta)
    wr, mur, covr, L0 = o4.em_step(X.astype(np.float64), *theta, 1e-3)
    e = mixture_errors((w, mu, cov), (wr, mur, covr), X)
    e["L0"] = abs(L[0] - L0) / max(abs(L0), X.shape[0])
    print(e, flush=True)
    assert max(e.values()) <= 1e-5, e
