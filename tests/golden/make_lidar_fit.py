"""Writes lidar_fit_oracle.npz: the FP64 oracle's fit of the synthetic LiDAR
scan (N = 2,000,000, K = 1000, T = 50 EM iterations, lambda = 1e-3, exact
two-pass centring), started from the oracle's k-means++ seeding with the
draws numpy.random.default_rng(1).random(1000).  Stored: the L history
(T + 1 values) and theta_T (w, mu, cov).  Calls the oracle only.

    python tests/golden/make_lidar_fit.py     (about 20 minutes on 8 cores)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2307_00071_amd import synth  # noqa: E402

K, T, REG = 1000, 50, 1e-3


def main():
    X = synth.lidar_scan(0)
    u = np.random.default_rng(1).random(K)
    _, lab = oracle.kmeanspp(X.astype(np.float64), K, u)
    w, mu, cov, L = oracle.fit(X, K, REG, T, labels=lab)
    np.savez_compressed(os.path.join(HERE, "lidar_fit_oracle.npz"), w=w, mu=mu, cov=cov,
                        L=L, K=K, T=T, reg=REG)
    print("L_T = %.9f" % L[-1])


if __name__ == "__main__":
    main()
