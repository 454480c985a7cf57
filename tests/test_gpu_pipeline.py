"""The paper's GPU pipeline end to end (the information-flow figure of Sec.
V: bandwidth and point cloud -> mean shift -> K -> KInit -> EM), every stage
on the GPU through the C ABI, against the same chain of oracles: the mean
shift's K, the k-means++ labels (same draws) and the 4D fit's log-likelihood
at every iteration (1e-4, floor N).  A subsample of the 320 x 240
depth-intensity frame keeps the oracle chain to seconds."""
import numpy as np
import pytest
import torch

import oracle
from oracle import gbms as og
from oracle import gmm4 as o4
import paper_2307_00071_amd as gmm
from paper_2307_00071_amd import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("n,h", [(4000, 0.3), (6000, 0.25)])
def test_meanshift_kinit_em4_chain(n, h):
    print("case: pipeline n=%d h=%g" % (n, h), flush=True)
    X = synth.depth_intensity_frame(0).reshape(480, 640, 4)[::2, ::2].reshape(-1, 4)
    rng = np.random.default_rng(9)
    X = np.ascontiguousarray(X[np.sort(rng.choice(X.shape[0], n, replace=False))])
    pts = torch.from_numpy(X).to(DEV)
    # mean shift: K
    _, _, info = gmm.meanshift(pts, h)
    K = info["n_modes"]
    om, _, _ = og.gbms(X.astype(np.float64), h)
    assert K == om.shape[0], (K, om.shape[0])
    assert 1 <= K <= 512
    # k-means++ on the xyz part (the same draws on both sides)
    u = np.random.default_rng(1).random(K)
    lab, cen = gmm.kmeanspp(pts[:, :3].contiguous(), K, u=u)
    torch.cuda.synchronize()
    rc, rl = oracle.kmeanspp(np.ascontiguousarray(X[:, :3]).astype(np.float64), K, u)
    np.testing.assert_array_equal(cen.cpu().numpy(), rc)
    np.testing.assert_array_equal(lab.cpu().numpy(), rl)
    # 4D EM from those labels
    T = 15
    r = gmm.fit4(pts, K, iters=T, labels=lab)
    torch.cuda.synchronize()
    L = r.loglik.cpu().numpy()
    Lr = o4.fit(X.astype(np.float64), K, 1e-3, T, labels=rl)[3]
    err = np.abs(L - Lr) / np.maximum(np.abs(Lr), n)
    assert err.max() <= 1e-4, err.max()
