"""GPU parity of distribution-to-distribution registration of two mixtures
(gmm_d2d_objective, gmm_d2d_register, through the C ABI) against the FP64
oracle (oracle/d2d.py).

Both sides compute in FP64 from the same float32 mixtures; they differ in
the order of the sums (the GPU's fixed block order against numpy's), the
form of the log-determinant and the log-sum-exp.  Bars:
  * f within 1e-12 max(1, |f|); the gradient element by element within
    1e-9 relative with a floor of 1e-10 max|grad| (entries that are sums of
    cancelling pair terms are judged on the gradient's scale);
  * registration: the same accepted iterations per stage, the history of f
    within 1e-11 max(1, |f|) entry by entry, the final transform within
    1e-9.  The step's accept test compares f between poses, so a decision
    could differ only where two values of f agree to about 1e-15; the
    stage stops before steps that small (max |x| < 1e-8).
Mixtures: random anisotropic ones, and mixtures the oracle fits to two
renders of the synthetic depth frame (the second with its own range noise,
moved by a known pose), the registration workload of the paper's Sec. IV at
K = 100 and K = 1000 (the full-size case compares the objective and
gradient with the oracle and checks the registration by its properties:
f never decreases, the counts are within budget, the gradient is small at
the end).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import d2d as od
import paper_2307_00071_amd as gmm
from paper_2307_00071_amd import _lib, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _case(name):
    print("case:", name, flush=True)


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
    return _f32(w, mu, cov)


def _f32(w, mu, cov):
    """float32 values (what the GPU reads), returned as float64 arrays."""
    cov = 0.5 * (cov + np.transpose(cov, (0, 2, 1)))
    return tuple(np.asarray(a, np.float32).astype(np.float64) for a in (w, mu, cov))


def _dev(mix):
    return tuple(torch.from_numpy(np.asarray(a, np.float32)).to(DEV) for a in mix)


def _moved(mix, R, t):
    w, mu, cov = mix
    return _f32(w, mu @ R.T + t, np.einsum("ab,kbc,dc->kad", R, cov, R))


_FRAME_CACHE = {}


def _frame_mixtures(K, n_sub=40000, iters=15):
    """Oracle fits of two renders of depth frame 0 (range noise from seeds
    None and 77); the second moved by random_pose(5)."""
    if K in _FRAME_CACHE:
        return _FRAME_CACHE[K]
    out = []
    pose = synth.random_pose(5, max_angle=0.15, max_trans=0.2)
    R = od.expso3(pose[:3])
    for noise in (None, 77):
        X = synth.depth_frame(0, noise_seed=noise) if noise else synth.depth_frame(0)
        rng = np.random.default_rng(3)
        X = X[np.sort(rng.choice(X.shape[0], n_sub, replace=False))].astype(np.float64)
        lab = synth.kmeanspp_labels(np.ascontiguousarray(X.astype(np.float32)), K, 1)
        w, mu, cov, _ = oracle.fit(X, K, 1e-3, iters, labels=lab)
        out.append((w, mu, cov))
    src = _f32(*out[0])
    tgt = _moved(_f32(*out[1]), R, pose[3:])
    _FRAME_CACHE[K] = (src, tgt, pose)
    return _FRAME_CACHE[K]


def _check_obj(pose, src, tgt, variant):
    f, g = gmm.d2d_objective(pose, _dev(src), _dev(tgt), variant=variant)
    if variant == "isoplanar":
        s2 = (src[0], src[1], od.isoplanar(src[2]))
        t2 = (tgt[0], tgt[1], od.isoplanar(tgt[2]))
    else:
        s2, t2 = src, tgt
    fo, go = od.objective_grad(np.asarray(pose, np.float64), s2, t2)
    assert abs(f - fo) <= 1e-12 * max(1.0, abs(fo)), (f, fo)
    den = 1e-9 * np.abs(go) + 1e-10 * np.abs(go).max()
    err = float((np.abs(g - go) / den).max())
    assert err <= 1.0, (g, go, err)
    return fo


@pytest.mark.parametrize("variant", ["anisotropic", "isoplanar"])
@pytest.mark.parametrize("m,n,seed", [(1, 1, 0), (5, 7, 1), (37, 64, 2), (300, 257, 3)])
def test_objective_and_gradient(variant, m, n, seed):
    _case("objective %s m=%d n=%d" % (variant, m, n))
    src = _mixture(seed, m)
    tgt = _mixture(seed + 50, n)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        pose = np.concatenate([rng.normal(0, 0.3, 3), rng.normal(0, 0.3, 3)])
        _check_obj(pose, src, tgt, variant)
    _check_obj(np.array([1e-6, -2e-6, 5e-7, 0.1, 0.0, 0.0]), src, tgt, variant)  # small angle


def _check_register(src, tgt, T0, iso, aniso):
    T, hist, counts = gmm.d2d_register(_dev(src), _dev(tgt), T0=T0, iters_iso=iso,
                                       iters_aniso=aniso)
    torch.cuda.synchronize()
    T, hist, counts = T.cpu().numpy(), hist.cpu().numpy(), counts.cpu().numpy()
    To, ho, co = od.register(T0, src, tgt, iters_iso=iso, iters_aniso=aniso)
    # the oracle lists the stages it ran; the GPU reports 0 for a skipped one
    got = [int(c) for c, it in zip(counts, (iso, aniso)) if it > 0]
    assert got == list(co), (counts, co)
    assert all(int(c) == 0 for c, it in zip(counts, (iso, aniso)) if it == 0)
    fo = np.array([f for _, f in ho])
    assert np.isnan(hist[len(fo):]).all()
    np.testing.assert_allclose(hist[:len(fo)], fo, rtol=0,
                               atol=1e-11 * max(1.0, np.abs(fo).max()))
    np.testing.assert_allclose(T, To, rtol=0, atol=1e-9)
    return T, hist, counts


@pytest.mark.parametrize("iso,aniso", [(0, 25), (15, 0), (10, 25)])
def test_register_random_mixtures(iso, aniso):
    _case("register random iso=%d aniso=%d" % (iso, aniso))
    src = _mixture(20, 12)
    Rs = od.expso3(np.array([0.12, -0.08, 0.18]))
    ts = np.array([0.15, -0.1, 0.12])
    tgt = _moved(_mixture(21, 15), Rs, ts)
    _check_register(src, tgt, np.eye(4), iso, aniso)


def test_register_recovers_a_rigid_motion():
    _case("register moved copy")
    src = _mixture(22, 20)
    Rs = od.expso3(np.array([0.15, -0.1, 0.2]))
    ts = np.array([0.2, -0.1, 0.15])
    tgt = _moved(src, Rs, ts)
    T, _, _ = _check_register(src, tgt, np.eye(4), 10, 40)
    # the moved copy's float32 rounding limits how exactly T* is the maximum
    np.testing.assert_allclose(T[:3, :3], Rs, atol=1e-5)
    np.testing.assert_allclose(T[:3, 3], ts, atol=1e-5)


def test_depth_frame_mixtures_k100():
    """The registration workload: mixtures of two renders of the depth frame
    (K = 100 each), the second moved by a known pose."""
    _case("depth-frame mixtures K=100")
    src, tgt, pose = _frame_mixtures(100)
    for variant in ("anisotropic", "isoplanar"):
        _check_obj(np.zeros(6), src, tgt, variant)
        _check_obj(pose, src, tgt, variant)
    T, hist, counts = _check_register(src, tgt, np.eye(4), 10, 30)
    R = od.expso3(pose[:3])
    print("pose error: rot %.2e rad, trans %.2e m; iterations %s" % (
        np.linalg.norm(T[:3, :3] - R), np.linalg.norm(T[:3, 3] - pose[3:]), counts), flush=True)


def test_depth_frame_mixtures_k1000_properties():
    """K = 1000 on each side (1e6 pairs): objective and gradient against the
    oracle at two poses; the registration by its properties."""
    _case("depth-frame mixtures K=1000")
    src, tgt, pose = _frame_mixtures(1000, n_sub=120000, iters=6)
    _check_obj(np.zeros(6), src, tgt, "anisotropic")
    _check_obj(pose, src, tgt, "anisotropic")
    T, hist, counts = gmm.d2d_register(_dev(src), _dev(tgt), iters_iso=10, iters_aniso=20)
    T, hist, counts = T.cpu().numpy(), hist.cpu().numpy(), counts.cpu().numpy()
    h = hist[~np.isnan(hist)]
    assert len(h) == counts.sum() + 2
    c0 = int(counts[0])
    assert np.all(np.diff(h[:1 + c0]) > 0)    # the isoplanar stage increases f
    assert np.all(np.diff(h[1 + c0:]) > 0)    # so does the anisotropic one
    Rt = T[:3, :3]
    np.testing.assert_allclose(Rt @ Rt.T, np.eye(3), atol=1e-12)
    pose_end = np.concatenate([_logso3(Rt), T[:3, 3]])
    f, g = od.objective_grad(pose_end, src, tgt)
    _, g0 = od.objective_grad(np.zeros(6), src, tgt)
    assert np.abs(g).max() <= 1e-2 * np.abs(g0).max() or counts[1] == 20


def _logso3(R):
    from scipy.spatial.transform import Rotation
    return Rotation.from_matrix(R).as_rotvec()


def test_bitwise_deterministic():
    _case("determinism")
    src = _mixture(30, 40)
    tgt = _mixture(31, 50)
    a = gmm.d2d_register(_dev(src), _dev(tgt), iters_iso=5, iters_aniso=10)
    b = gmm.d2d_register(_dev(src), _dev(tgt), iters_iso=5, iters_aniso=10)
    for x, y in zip(a, b):
        assert torch.equal(x, y) or (torch.isnan(x) == torch.isnan(y)).all() and \
            torch.equal(torch.nan_to_num(x), torch.nan_to_num(y))


def test_errors():
    _case("errors")
    src = _mixture(40, 4)
    tgt = _mixture(41, 5)
    bad = (src[0].copy(), src[1], src[2])
    bad[0][1] = 0.0
    with pytest.raises(_lib.GmmError) as e:
        gmm.d2d_objective(np.zeros(6), _dev(bad), _dev(tgt))
    assert e.value.status == _lib.GMM_ERR_INVALID_ARG
    nanm = (src[0], src[1].copy(), src[2])
    nanm[1][0, 0] = np.nan
    with pytest.raises(_lib.GmmError) as e:
        gmm.d2d_objective(np.zeros(6), _dev(nanm), _dev(tgt))
    assert e.value.status == _lib.GMM_ERR_NONFINITE
    with pytest.raises(KeyError):
        gmm.d2d_objective(np.zeros(6), _dev(src), _dev(tgt), variant="planar")
    lib = _lib.load()
    assert lib.gmm_d2d_workspace_size(0, 5) == 0
    # the library still works afterwards
    _check_obj(np.zeros(6), src, tgt, "anisotropic")


def test_graph_replay_is_bitwise_equal_to_direct_launches():
    """The same C-ABI registration three times with the same buffers: the
    first runs its kernels directly, the second captures them into a graph,
    the third replays it; all three give the same bits, and the graph reads
    the inputs' current contents (a fourth call after the target moved
    matches a direct call on the moved target)."""
    import ctypes
    _case("d2d graph replay")
    src = _mixture(50, 60)
    R = _rot(0.1, 0.05, -0.08)
    tgt = _moved(src, R, np.array([0.1, -0.05, 0.08]))
    lib = _lib.load()
    s = _dev(src)
    t = [x.clone() for x in _dev(tgt)]
    T0 = torch.eye(4, dtype=torch.float64, device=DEV)
    T = torch.empty(4, 4, dtype=torch.float64, device=DEV)
    iso, aniso = 5, 10
    hist = torch.empty(iso + aniso + 2, dtype=torch.float64, device=DEV)
    counts = torch.empty(2, dtype=torch.int32, device=DEV)
    m, n = s[0].shape[0], t[0].shape[0]
    ws = torch.empty(lib.gmm_d2d_workspace_size(m, n), dtype=torch.uint8, device=DEV)
    stream = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    p = lambda x: ctypes.c_void_p(x.data_ptr())

    def call():
        _lib.check(lib.gmm_d2d_register(p(T0), m, p(s[0]), p(s[1]), p(s[2]), n, p(t[0]),
                                        p(t[1]), p(t[2]), iso, aniso, p(T), p(hist), p(counts),
                                        p(ws), ws.numel(), stream))
        torch.cuda.synchronize()
        return [x.cpu().numpy().copy() for x in (T, hist, counts)]

    outs = [call() for _ in range(3)]
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            np.testing.assert_array_equal(a, b)
    # move the target in place: the replayed graph sees the new values
    tgt2 = _moved(src, _rot(-0.05, 0.1, 0.02), np.array([-0.1, 0.0, 0.05]))
    for dst, x in zip(t, _dev(tgt2)):
        dst.copy_(x)
    replay = call()
    direct = [x.cpu().numpy() for x in gmm.d2d_register(_dev(src), _dev(tgt2), iters_iso=iso,
                                                         iters_aniso=aniso)]
    for a, b in zip(replay, direct):
        np.testing.assert_array_equal(a, b)


def _rot(a, b, c):
    from scipy.spatial.transform import Rotation
    return Rotation.from_rotvec([a, b, c]).as_matrix()
