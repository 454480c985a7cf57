"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module generates point clouds, initial hard labels and poses.  It holds
none of the EM arithmetic (no responsibilities, no statistics, no
Cholesky), imports nothing else from this package and nothing from the
oracle, so both sides can use it without sharing method code.

Workloads (all float32, metres):

* ``gaussian_blobs``  - 8 anisotropic Gaussians, means in a 10 m cube,
  Sigma = R diag(s)^2 R^T with Haar-random R and s ~ U[0.05, 0.5], exactly
  1250 points each (10,000 points).
* ``depth_frame``     - a 640x480 pinhole depth frame (fx = fy = 525,
  cx = 319.5, cy = 239.5, z forward) cast into a closed room box holding
  6-12 random planar patches and oriented boxes at 0.5-8 m, with Gaussian
  range noise along each ray; every ray hits, so N = 307,200.  It stands
  in for the indoor RGB-D frames the paper evaluates on.
* ``depth_intensity_frame`` - the same frame with a per-point intensity
  (per-surface albedo, a smooth positional texture and noise): the 4D
  (x, y, z, intensity) cloud of the paper's model.
* ``batched_frames``  - 64 depth frames (seeds 1000+f) subsampled to
  N_f ~ U{20000..300000}, each with K_f ~ U{16..200}.
* ``lidar_scan``      - a 64-ring spinning scan (elevation -25..+15 deg,
  0.2 deg azimuth step) of a ground plane, vertical walls and vertical
  cylinders out to 80 m, 0.02 m range noise, accumulated over sweeps along
  a short trajectory and cut to exactly N points.
* ``kmeanspp_labels`` - the random initialisation (k-means++ D^2 seeding,
  one trial per centre, then each point labelled with its nearest seed,
  ties to the lowest index).  EM's first M-step turns these one-hot
  responsibilities into theta_0.
* ``random_pose``     - axis-angle rotation of at most 0.3 rad and a
  translation of at most 0.5 m.
"""
from __future__ import annotations

import numpy as np


def haar_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random rotation: QR of a Gaussian matrix with the sign fix,
    then a determinant fix so the result is proper."""
    A = rng.standard_normal((3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def gaussian_blobs(seed: int = 0, n_per: int = 1250, k: int = 8,
                   cube: float = 10.0, smin: float = 0.05, smax: float = 0.5):
    """Points from k anisotropic Gaussians with equal counts (no multinomial
    noise).  Returns (X float32 (k*n_per, 3), generating means, covs)."""
    rng = np.random.default_rng(seed)
    X = np.empty((k * n_per, 3))
    means = np.empty((k, 3))
    covs = np.empty((k, 3, 3))
    for b in range(k):
        mu = rng.uniform(0.0, cube, 3)
        R = haar_rotation(rng)
        s = rng.uniform(smin, smax, 3)
        z = rng.standard_normal((n_per, 3))
        X[b * n_per:(b + 1) * n_per] = mu + (z * s) @ R.T
        means[b] = mu
        covs[b] = R @ np.diag(s * s) @ R.T
    return X.astype(np.float32), means, covs


# ---------------------------------------------------------------- ray casting

def _ray_obb(o, d, center, R, half):
    """Nearest positive hit distance of rays (o, d) with an oriented box;
    inf where missed.  Slab test in the box frame."""
    ol = (o - center) @ R          # (3,) or (N,3)
    dl = d @ R
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (-half - ol) / dl
        t2 = (half - ol) / dl
    tlo = np.nanmax(np.minimum(t1, t2), axis=1)
    thi = np.nanmin(np.maximum(t1, t2), axis=1)
    hit = (thi >= tlo) & (tlo > 1e-6)
    return np.where(hit, tlo, np.inf)


def _ray_rect(o, d, center, normal, e1, e2, h1, h2):
    """Nearest positive hit distance with a planar rectangle."""
    den = d @ normal
    with np.errstate(divide="ignore", invalid="ignore"):
        t = ((center - o) @ normal) / den
    p = o + t[:, None] * d - center
    ok = (t > 1e-6) & (np.abs(p @ e1) <= h1) & (np.abs(p @ e2) <= h2)
    return np.where(ok, t, np.inf)


def _ray_vcyl(o, d, cxy, r, z0, z1):
    """Nearest positive hit distance with a vertical cylinder (z up)."""
    ox = o[..., 0] - cxy[0]
    oy = o[..., 1] - cxy[1]
    a = d[:, 0] ** 2 + d[:, 1] ** 2
    b = 2.0 * (ox * d[:, 0] + oy * d[:, 1])
    c = ox * ox + oy * oy - r * r
    disc = b * b - 4 * a * c
    with np.errstate(divide="ignore", invalid="ignore"):
        sq = np.sqrt(np.maximum(disc, 0.0))
        ta = (-b - sq) / (2 * a)
        tb = (-b + sq) / (2 * a)
    t = np.where(ta > 1e-6, ta, tb)
    z = o[..., 2] + t * d[:, 2]
    ok = (disc >= 0) & (a > 0) & (t > 1e-6) & (z >= z0) & (z <= z1)
    return np.where(ok, t, np.inf)


def _depth_render(seed, width, height, fx, fy, cx, cy, sigma, noise_seed):
    """Ray casting of one synthetic scene: (points float64 (N, 3), id of the
    surface each ray hit: 0..5 the room's faces, 6 + j object j)."""
    rng = np.random.default_rng(seed)
    u, v = np.meshgrid(np.arange(width, dtype=np.float64),
                       np.arange(height, dtype=np.float64))
    d = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], -1)
    d = d.reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.zeros(3)
    # enclosing room (axis-aligned box around the camera)
    lo = np.array([-rng.uniform(2.5, 4.0), -rng.uniform(1.0, 1.6), -1.0])
    hi = np.array([rng.uniform(2.5, 4.0), rng.uniform(1.2, 1.8),
                   rng.uniform(6.5, 8.0)])
    with np.errstate(divide="ignore", invalid="ignore"):
        tw = np.where(d > 0, hi / d, np.where(d < 0, lo / d, np.inf))
    t = tw.min(axis=1)
    face = tw.argmin(axis=1) * 2 + (d[np.arange(d.shape[0]), tw.argmin(axis=1)] > 0)
    hit = face.astype(np.int64)
    n_obj = int(rng.integers(6, 13))
    for j in range(n_obj):
        # place the object centre along a random in-frustum ray at 0.5-8 m
        px, py = rng.uniform(0, width), rng.uniform(0, height)
        ray = np.array([(px - cx) / fx, (py - cy) / fy, 1.0])
        ray /= np.linalg.norm(ray)
        depth = rng.uniform(0.8, 7.0)
        center = o + depth * ray
        R = haar_rotation(rng)
        if rng.uniform() < 0.5:
            half = rng.uniform(0.1, 0.8, 3)
            th = _ray_obb(o, d, center, R, half)
        else:
            th = _ray_rect(o, d, center, R[:, 2], R[:, 0], R[:, 1],
                           rng.uniform(0.2, 1.2), rng.uniform(0.2, 1.2))
        hit = np.where(th < t, 6 + j, hit)
        t = np.minimum(t, th)
    assert np.all(np.isfinite(t))
    nrng = rng if noise_seed is None else np.random.default_rng(noise_seed)
    t = t + sigma * nrng.standard_normal(t.shape)
    return t[:, None] * d, hit


def depth_frame(seed: int = 0, width: int = 640, height: int = 480,
                fx: float = 525.0, fy: float = 525.0, cx: float = 319.5,
                cy: float = 239.5, sigma: float = 0.01,
                noise_seed=None) -> np.ndarray:
    """One synthetic depth frame in the camera frame (x right, y down,
    z forward).  Returns float32 (width*height, 3); every ray hits.
    ``noise_seed`` (optional) draws the range noise from its own generator:
    a second noisy render of the same scene."""
    pts, _ = _depth_render(seed, width, height, fx, fy, cx, cy, sigma, noise_seed)
    return pts.astype(np.float32)


def depth_intensity_frame(seed: int = 0, width: int = 640, height: int = 480,
                          sigma_i: float = 0.02) -> np.ndarray:
    """The depth frame of ``depth_frame(seed)`` with an intensity channel:
    float32 (N, 4) = (x, y, z, intensity).  Each surface has its own albedo
    U[0.15, 0.85], modulated by a smooth texture 0.1 sin(2.3 x) cos(1.7 y)
    + 0.05 sin(3.1 z) of the position and N(0, sigma_i^2) noise (the
    points are exactly those of depth_frame(seed); the intensities come
    from generators of their own).  It stands in for the depth-intensity
    image pairs the paper models."""
    pts, hit = _depth_render(seed, width, height, 525.0, 525.0, 319.5, 239.5,
                             0.01, None)
    rng = np.random.default_rng(seed + 7919)
    albedo = rng.uniform(0.15, 0.85, int(hit.max()) + 1)
    tex = (0.1 * np.sin(2.3 * pts[:, 0]) * np.cos(1.7 * pts[:, 1])
           + 0.05 * np.sin(3.1 * pts[:, 2]))
    inten = albedo[hit] + tex + sigma_i * rng.standard_normal(pts.shape[0])
    return np.concatenate([pts, inten[:, None]], axis=1).astype(np.float32)


def batched_frames(seed_base: int = 1000, count: int = 64, nmin: int = 20000,
                   nmax: int = 300000, kmin: int = 16, kmax: int = 200):
    """Uneven frames for batched fitting: list of (X_f float32, K_f)."""
    out = []
    for f in range(count):
        rng = np.random.default_rng(seed_base + f)
        n_f = int(rng.integers(nmin, nmax + 1))
        k_f = int(rng.integers(kmin, kmax + 1))
        X = depth_frame(seed=seed_base + f)
        idx = rng.choice(X.shape[0], size=n_f, replace=False)
        out.append((np.ascontiguousarray(X[np.sort(idx)]), k_f))
    return out


def lidar_scan(seed: int = 0, n_points: int = 2_000_000, rings: int = 64,
               el_lo: float = -25.0, el_hi: float = 15.0, az_step: float = 0.2,
               max_range: float = 80.0, sigma: float = 0.02,
               sensor_height: float = 1.8) -> np.ndarray:
    """Accumulated spinning-LiDAR sweeps in a world frame (z up)."""
    rng = np.random.default_rng(seed)
    el = np.deg2rad(np.linspace(el_lo, el_hi, rings))
    n_az = int(round(360.0 / az_step))
    walls = []
    for _ in range(int(rng.integers(20, 36))):
        ang = rng.uniform(0, 2 * np.pi)
        dist = rng.uniform(5.0, max_range - 5.0)
        c = np.array([dist * np.cos(ang), dist * np.sin(ang), 0.0])
        yaw = rng.uniform(0, np.pi)
        nrm = np.array([np.cos(yaw), np.sin(yaw), 0.0])
        e1 = np.array([-np.sin(yaw), np.cos(yaw), 0.0])
        hgt = rng.uniform(2.0, 12.0)
        c[2] = -sensor_height + hgt / 2
        walls.append((c, nrm, e1, np.array([0.0, 0.0, 1.0]),
                      rng.uniform(2.0, 15.0), hgt / 2))
    cyls = []
    for _ in range(int(rng.integers(20, 41))):
        ang = rng.uniform(0, 2 * np.pi)
        dist = rng.uniform(3.0, max_range - 3.0)
        cyls.append((np.array([dist * np.cos(ang), dist * np.sin(ang)]),
                     rng.uniform(0.1, 1.0), -sensor_height,
                     -sensor_height + rng.uniform(1.0, 10.0)))
    pts = []
    total = 0
    sweep = 0
    while total < n_points:
        pos = np.array([0.6 * sweep, 0.15 * np.sin(0.3 * sweep), 0.0])
        phase = rng.uniform(0, az_step)
        az = np.deg2rad(phase + az_step * np.arange(n_az))
        E, A = np.meshgrid(el, az, indexing="ij")
        d = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A),
                      np.sin(E)], -1).reshape(-1, 3)
        with np.errstate(divide="ignore", invalid="ignore"):
            tg = np.where(d[:, 2] < 0, (-sensor_height - pos[2]) / d[:, 2],
                          np.inf)
        t = tg
        for (c, nrm, e1, e2, h1, h2) in walls:
            t = np.minimum(t, _ray_rect(pos, d, c, nrm, e1, e2, h1, h2))
        for (cxy, r, z0, z1) in cyls:
            t = np.minimum(t, _ray_vcyl(pos, d, cxy, r, z0, z1))
        keep = t <= max_range
        t = t[keep] + sigma * rng.standard_normal(int(keep.sum()))
        P = pos + t[:, None] * d[keep]
        pts.append(P.astype(np.float32))
        total += P.shape[0]
        sweep += 1
    return np.concatenate(pts, axis=0)[:n_points]


# --------------------------------------------------------- initialisation

def kmeanspp_labels(X: np.ndarray, K: int, seed: int) -> np.ndarray:
    """k-means++ D^2 seeding (one trial per centre) and nearest-seed labels.

    The first seed is a uniformly random point; each later seed is drawn
    with probability proportional to the squared distance to the nearest
    seed chosen so far.  Labels are the index of the nearest seed, ties to
    the lowest index.  Distances are computed in float64."""
    rng = np.random.default_rng(seed)
    Xd = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    N = Xd.shape[0]
    if not 0 < K <= N:
        raise ValueError("need 0 < K <= N")
    cols = [np.ascontiguousarray(Xd[:, j]) for j in range(3)]
    tmp = np.empty(N)
    dist = np.empty(N)

    def sqdist(idx):
        np.subtract(cols[0], cols[0][idx], out=tmp)
        np.multiply(tmp, tmp, out=dist)
        for j in (1, 2):
            np.subtract(cols[j], cols[j][idx], out=tmp)
            np.multiply(tmp, tmp, out=tmp)
            np.add(dist, tmp, out=dist)
        return dist

    first = int(rng.integers(N))
    best = sqdist(first).copy()
    labels = np.zeros(N, dtype=np.int32)
    cdf = np.empty(N)
    closer = np.empty(N, dtype=bool)
    for k in range(1, K):
        np.cumsum(best, out=cdf)
        if cdf[-1] > 0:
            idx = int(np.searchsorted(cdf, rng.uniform() * cdf[-1], side="right"))
            idx = min(idx, N - 1)
        else:
            idx = int(rng.integers(N))
        d = sqdist(idx)
        np.less(d, best, out=closer)
        labels[closer] = k
        np.minimum(best, d, out=best)
    return labels


def random_pose(seed: int, max_angle: float = 0.3, max_trans: float = 0.5):
    """pose6 = (omega, t): random unit axis times U[0, max_angle] rad and a
    random unit direction times U[0, max_trans] m (float64)."""
    rng = np.random.default_rng(seed)
    ax = rng.standard_normal(3)
    ax /= np.linalg.norm(ax)
    tr = rng.standard_normal(3)
    tr /= np.linalg.norm(tr)
    return np.concatenate([ax * rng.uniform(0, max_angle),
                           tr * rng.uniform(0, max_trans)])


def random_theta(K: int, seed: int, spread: float = 5.0, smin: float = 0.1,
                 smax: float = 1.0):
    """A random valid mixture (w normalised, SPD covariances) for tests of
    single E/M steps (float64)."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.2, 1.0, K)
    w /= w.sum()
    mu = rng.uniform(-spread, spread, (K, 3))
    cov = np.empty((K, 3, 3))
    for b in range(K):
        R = haar_rotation(rng)
        s = rng.uniform(smin, smax, 3)
        cov[b] = R @ np.diag(s * s) @ R.T
        cov[b] = 0.5 * (cov[b] + cov[b].T)
    return w, mu, cov
