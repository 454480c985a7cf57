"""GPU k-means++ seeding (gmm_kmeanspp through the C ABI) against the
definition and the oracle.

The GPU turns a draw into an index through chunked running sums (256
points per chunk, chunk totals in runs of 16 from block-scan offsets, a
block scan inside the chosen chunk); the oracle through one flat running
sum.  Floating-point running sums depend on their order, so the two may
part only where u_j W lies within rounding of a running sum.  Every GPU
seeding is therefore checked along its own trajectory against the exact
running sums of the same double-precision D2 (tests/kpp_check.py: every
pick is valid up to the GPU's own rounding budget), its labels are
compared bit for bit with the oracle's nearest-centre labels of the GPU's
centres, and its centres with the oracle's seeding up to the first
certified tie (none occurs on these inputs, so the full sequences are
compared)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_00071_amd as gmm
from paper_2307_00071_amd import _lib, synth
from tests.kpp_check import check_trajectory, gpu_sum_terms

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _case(name):
    print("case:", name, flush=True)


def _both(X, K, u, validate=True):
    """GPU seeding and the oracle's.  With `validate`, the GPU's picks are
    checked along their own trajectory and its labels against the oracle's
    nearest centres of the GPU's centres; the returned oracle centres are
    cut to agree after a certified tie (the trajectories then part)."""
    Xf = np.ascontiguousarray(X, dtype=np.float32)
    lab, cen = gmm.kmeanspp(torch.from_numpy(Xf).to(DEV), K, u=u)
    torch.cuda.synchronize()
    X64 = Xf.astype(np.float64)
    cen, lab = cen.cpu().numpy(), lab.cpu().numpy()
    rc, rl = oracle.kmeanspp(X64, K, u)
    if validate:
        ties = check_trajectory(X64, u, cen, gpu_sum_terms(X64.shape[0]))
        np.testing.assert_array_equal(lab, oracle.nearest(X64, cen))
        if ties:
            print("certified ties at steps", ties, flush=True)
            rc = np.concatenate([rc[:ties[0]], cen[ties[0]:]])
            rl = lab
    return cen, lab, rc, rl


def _depth_subset(n, seed):
    X = synth.depth_frame(seed)
    rng = np.random.default_rng(seed + 5)
    return np.ascontiguousarray(X[np.sort(rng.choice(X.shape[0], n, replace=False))])


CASES = [
    ("blobs", 10000, 8), ("int-cloud", 20000, 12), ("depth-ragged", 16385, 37),
    ("depth-ragged", 257, 257), ("depth-ragged", 300, 1), ("one-point", 1, 1),
    ("depth-ragged", 70001, 150),
]


@pytest.mark.parametrize("kind,n,K", CASES)
def test_kmeanspp_matches_oracle(kind, n, K):
    _case("kmeanspp %s n=%d K=%d" % (kind, n, K))
    if kind == "blobs":
        X = synth.gaussian_blobs(0, n_per=n // 8)[0]
    elif kind == "int-cloud":
        X = np.random.default_rng(3).integers(0, 40, (n, 3)).astype(np.float32)
    elif kind == "one-point":
        X = np.array([[0.5, -1.0, 2.0]], dtype=np.float32)
    else:
        X = _depth_subset(n, seed=K)
    u = np.random.default_rng(n + K).random(K)
    cen, lab, rc, rl = _both(X, K, u)
    np.testing.assert_array_equal(cen, rc)
    np.testing.assert_array_equal(lab, rl)


def test_kmeanspp_depth_frame_full():
    _case("kmeanspp depth frame N=307200 K=100")
    X = synth.depth_frame(0)
    u = np.random.default_rng(1).random(100)
    cen, lab, rc, rl = _both(X, 100, u)
    np.testing.assert_array_equal(cen, rc)
    np.testing.assert_array_equal(lab, rl)


def test_kmeanspp_lidar_scan_full():
    _case("kmeanspp lidar N=2000000 K=1000")
    X = synth.lidar_scan(0)
    u = np.random.default_rng(1).random(1000)
    cen, lab, rc, rl = _both(X, 1000, u)
    np.testing.assert_array_equal(cen, rc)
    np.testing.assert_array_equal(lab, rl)


def test_kmeanspp_more_groups_than_one_stage():
    """n > 16,384 chunks of 256 points: the chunk totals are scanned in
    stages (the staged search path)."""
    _case("kmeanspp n=17000000 K=4")
    X = np.random.default_rng(8).uniform(-50, 50, (17_000_000, 3)).astype(np.float32)
    u = np.array([0.3, 0.999, 0.5, 0.01])
    cen, lab, rc, rl = _both(X, 4, u)
    np.testing.assert_array_equal(cen, rc)
    np.testing.assert_array_equal(lab, rl)


def test_kmeanspp_degenerate_inputs():
    _case("kmeanspp degenerate")
    X = np.tile(np.array([[1.5, -2.0, 3.25]], dtype=np.float32), (600, 1))
    cen, lab, rc, rl = _both(X, 5, np.array([0.3, 0.1, 0.9, 0.5, 0.0]))
    np.testing.assert_array_equal(cen, rc)
    assert (cen == cen[0]).all() and not lab.any()
    X = _depth_subset(5000, 9)
    X[:2000] = X[0]
    u = np.array([0.0, 0.0, 1.0 - 2.0 ** -53, 0.5, 1.0 - 2.0 ** -53, 0.25])
    cen, lab, rc, rl = _both(X, 6, u)
    np.testing.assert_array_equal(cen, rc)
    np.testing.assert_array_equal(lab, rl)


def test_kmeanspp_reports_bad_draws_and_points():
    _case("kmeanspp errors")
    X = torch.from_numpy(_depth_subset(1000, 2)).to(DEV)
    with pytest.raises(_lib.GmmError) as e:
        gmm.kmeanspp(X, 4, u=np.array([0.1, 0.2, 1.0, 0.3]))
    assert e.value.status == 1
    Xn = X.clone()
    Xn[17, 2] = float("nan")
    with pytest.raises(_lib.GmmError) as e:
        gmm.kmeanspp(Xn, 4, seed=0)
    assert e.value.status == 3
    with pytest.raises(_lib.GmmError) as e:
        gmm.kmeanspp(X[:3], 4, seed=0)
    assert e.value.status == 1


def test_kmeanspp_then_fit_matches_oracle():
    """GPU seeding feeds the GPU fit; the oracle fits from its own seeding
    of the same draws (identical labels), final L within the fit bar."""
    _case("kmeanspp then fit")
    X = _depth_subset(30000, 4)
    K, T = 40, 20
    Xt = torch.from_numpy(X).to(DEV)
    lab, _ = gmm.kmeanspp(Xt, K, seed=7)
    r = gmm.fit(Xt, K, iters=T, reg_covar=1e-3, labels=lab)
    torch.cuda.synchronize()
    _, rl = oracle.kmeanspp(X.astype(np.float64), K, np.random.default_rng(7).random(K))
    np.testing.assert_array_equal(lab.cpu().numpy(), rl)
    Lo = oracle.fit(X, K, 1e-3, T, labels=rl)[3]
    Lg = r.loglik.cpu().numpy()
    assert abs(Lg[-1] - Lo[-1]) <= 1e-4 * max(abs(Lo[-1]), X.shape[0])


def test_kmeanspp_without_labels_through_the_abi():
    """labels = NULL: centres only (equal to the oracle's); with K = 1 the
    points are still checked for non-finite values."""
    import ctypes
    _case("kmeanspp labels NULL")
    lib = _lib.load()
    X = _depth_subset(5000, 3)
    Xt = torch.from_numpy(X).to(DEV)
    u = np.random.default_rng(4).random(6)
    ut = torch.from_numpy(u).to(DEV)
    cen = torch.empty(6, dtype=torch.int64, device=DEV)
    st = lib.gmm_kmeanspp(ctypes.c_void_p(Xt.data_ptr()), 5000, 6,
                          ctypes.c_void_p(ut.data_ptr()), ctypes.c_void_p(cen.data_ptr()),
                          None, None, 0, None)
    assert st == 0
    rc, _ = oracle.kmeanspp(X.astype(np.float64), 6, u)
    np.testing.assert_array_equal(cen.cpu().numpy(), rc)
    Xn = Xt.clone()
    Xn[4321, 0] = float("inf")
    st = lib.gmm_kmeanspp(ctypes.c_void_p(Xn.data_ptr()), 5000, 1,
                          ctypes.c_void_p(ut.data_ptr()), ctypes.c_void_p(cen.data_ptr()),
                          None, None, 0, None)
    assert st == 3
