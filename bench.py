"""Benchmark: EM fitting of a 3D GMM to a synthetic 640x480 depth frame.

Workload: N = 307,200 points (640x480 pinhole rays cast into a random room
with 6-12 planes/boxes, 0.01 m range noise), K = 100, T = 100 EM
iterations from k-means++ hard labels, lambda = 1e-3 m^2.  One step = one
full gmm_fit call (label M-step, T E+M iterations, final log-likelihood),
points already resident in HBM.

Prints one JSON line:
  value           point-component evals/s = N*K*T / (time per fit), fits
                  replayed as captured hipGraphs (the library's default for
                  repeated calls)
  em_iters_per_s  T / (time per fit)
  roofline        the E+M tile kernel: algorithmic FLOP per launch
                  (42 FLOP per point-component evaluation) / its mean
                  duration from HIP events on the fit's stream, over a
                  second timed region of the same fits with direct launches
                  (HIP does not time events inside a replayed graph); each
                  pair brackets 16 back-to-back launches of the same
                  (idempotent) tile pass, so the pair's own dispatch latency
                  is spread over 16 launches
  batched         64 uneven depth frames (N_f ~ U[20k, 300k], K_f ~ U[16,
                  200]) fitted by one gmm_fit_batched call vs 64 sequential
                  gmm_fit calls (direct launches), same T
  lidar           the large fit: a synthetic 64-ring LiDAR scan, N =
                  2,000,000, K = 1000, T = 50, two-pass FP64 moments (and
                  shifted one-pass moments for comparison), started from the
                  GPU k-means++ seeding
  kinit           k-means++ seeding on the GPU (gmm_kmeanspp) at the depth
                  frame (K = 100) and the LiDAR scan (K = 1000), beside the
                  oracle's seeding of the same draws on the host cores
  blobs           the small fit: N = 10,000 points from 8 anisotropic
                  Gaussians, K = 8, T = 50, GPU k-means++ seeding:
                  microseconds per EM iteration (launch-latency bound)
  registration    log-likelihood of a moved cloud (N = 100,000) under a
                  fitted K = 200 mixture, its forward and backward kernels
                  and the gradient with respect to pose, points and
                  mixture; roofline of the backward tile kernel; the
                  oracle's likelihood + gradient on the host beside it
  cpu_baseline    the FP64 CPU oracle on a bounded sample of the same fit
                  (all host cores); cpu_baseline_1thread the same on one
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("EM iters/s and point-component evals/s at N=307200,K=100; "
          "batched vs plain")
FLOP_PER_EVAL = 42          # distance 19 + log-sum-exp 3 + statistics 20
FLOP_PER_EVAL_FWD = 22      # registration forward: distance 19 + log-sum-exp 3
FLOP_PER_EVAL_BWD = 57      # backward: forward 22 + gradient terms 15 + statistics 20
PEAK_FP32_VECTOR = 157.3    # TFLOP/s, MI355X FP32 vector (packed FMA rate)
PEAK_FP64_VECTOR = 78.6     # TFLOP/s, MI355X FP64 vector
FLOP_PER_EVAL_4D = 76       # 4D: E-step 34, log-sum-exp 3, statistics 39
D2D_FLOP_VALUE = 45         # FP64 per pair term of a D2D value pass
D2D_FLOP_STATS = 290        # FP64 per pair term of the D2D statistics pass
PEAK_FP32_NONPACKED = 78.6  # TFLOP/s, one FP32 FMA per lane per cycle
PROFILE_REPS = 16           # tile launches per timed event pair

# HBM traffic of one E+M tile launch at this workload, from two rocprofv3
# --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch, averaged over
# the iteration launches), scaled by what the same counters read for a
# 256 MiB device copy (FETCH_SIZE reads half the bytes moved, WRITE_SIZE all
# of them).  Valid only for the kernel source and tile shape it was taken
# on: any other reports null.
TRAFFIC = {"kernel_src_sha256": "96378b2c16652575e51f12c8a29d9fe1d6925791e91d8cb443fda5f49bb14064",
           "tile_shape": "c512t128p16", "N": 307200, "K": 100,
           "fetch_kib": 2668.11, "fetch_factor": 2.0,
           "write_kib": 6044.21, "write_factor": 1.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target wall time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-iters", type=int, default=20)
    ap.add_argument("--no-lidar", action="store_true")
    ap.add_argument("--no-kinit", action="store_true")
    ap.add_argument("--no-blobs", action="store_true")
    ap.add_argument("--no-registration", action="store_true")
    ap.add_argument("--no-model4d", action="store_true")
    ap.add_argument("--no-pipeline", action="store_true")
    ap.add_argument("--no-meanshift", action="store_true")
    ap.add_argument("--no-d2d", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 256 MiB device-to-device tensor copy "
                         "(a known-size reference for memory counters)")
    return ap.parse_args()


def tile_traffic_bytes(N, K):
    """HBM bytes per tile launch from the recorded counters, or None when the
    kernel source, tile shape or workload differs from where they were taken."""
    import hashlib
    from paper_2307_00071_amd import _lib
    src = os.path.join(ROOT, "paper_2307_00071_amd", "csrc", "em_device.hpp")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    t = TRAFFIC
    if (sha != t["kernel_src_sha256"] or (N, K) != (t["N"], t["K"])
            or _lib.tile_config(N, K) != t["tile_shape"]):
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_factor"] +
                     t["write_kib"] * t["write_factor"])


def cpu_baseline(X, lab, K, T_hint, target_s, threads=None):
    """Time the FP64 oracle (as it stands) on a bounded number of EM
    iterations of the same fit; report evals/s."""
    import oracle
    prev = oracle.get_threads()
    if threads:
        oracle.set_threads(threads)
    threads = oracle.get_threads()
    N = X.shape[0]
    t0 = time.perf_counter()
    oracle.fit(X, K, 1e-3, 1, labels=lab)
    t1 = time.perf_counter() - t0
    iters = int(max(1, min(T_hint, round(target_s / max(t1, 1e-3)))))
    if iters == 1:
        dt = t1
    else:
        t0 = time.perf_counter()
        oracle.fit(X, K, 1e-3, iters, labels=lab)
        dt = time.perf_counter() - t0
    oracle.set_threads(prev)
    return {"value": N * K * iters / dt, "unit": "point-component evals/s",
            "cores": threads, "kind": "oracle",
            "sample": "%d EM iterations (label M-step + %d x (E-step + "
                      "two-pass M-step) + final E-step) of the same N=%d, "
                      "K=%d fit, FP64, %.1f s wall" % (iters, iters, N, K, dt)}


def batched_vs_plain(T, reps=2, single_evals_per_s=None):
    """64 uneven frames: one gmm_fit_batched call (soft-pass shape chosen by
    the library's autotuner on the first call) vs 64 gmm_fit calls."""
    import numpy as np
    import torch

    import paper_2307_00071_amd as gmm
    from paper_2307_00071_amd import _lib, synth

    dev = torch.device("cuda:0")
    frames = synth.batched_frames()
    pts = [torch.from_numpy(X).to(dev) for X, _ in frames]
    ks = [k for _, k in frames]
    ns = [X.shape[0] for X, _ in frames]
    labs = [torch.from_numpy(synth.kmeanspp_labels(X, k, 1)).to(dev)
            for X, k in frames]
    evals = sum(X.shape[0] * k for X, k in frames) * T
    ws = torch.empty(gmm.fit_batched_workspace_bytes(ns, ks, T),
                     dtype=torch.uint8, device=dev)

    def batched():
        return gmm.fit_batched(pts, ks, iters=T, labels_list=labs, workspace=ws)

    def plain():
        return [gmm.fit(p, k, iters=T, labels=l) for p, k, l in zip(pts, ks, labs)]

    out = {}
    _lib.set_autotune(True)
    try:
        batched()                      # tunes the soft-pass shape
        torch.cuda.synchronize()
        out["shape"] = _lib.batch_config(ns, ks)
        for name, fn in (("batched", batched), ("plain", plain)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                res = fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            out[name + "_ms"] = 1e3 * dt
            out[name + "_evals_per_s"] = evals / dt
            out[name + "_final_loglik_sum"] = float(sum(r.loglik[-1].item() for r in res))
        # soft-pass kernel time of the batched fit (direct launches)
        _lib.profile_read()
        _lib.profile_pairs()
        _lib.profile_enable(PROFILE_REPS)
        batched()
        torch.cuda.synchronize()
        _lib.profile_enable(0)
        ms, n = _lib.profile_read()
        _lib.profile_pairs()
    finally:
        _lib.set_autotune(False)
    avg = ms / max(n, 1) * 1e-3
    ach = FLOP_PER_EVAL * (evals / T) / avg / 1e12
    out["roofline"] = {"bound": "alu", "kernel": "batched soft pass, shape %s" % out["shape"],
                       "achieved": ach, "peak": PEAK_FP32_VECTOR, "unit": "TFLOP/s",
                       "frac": ach / PEAK_FP32_VECTOR, "avg_launch_us": 1e6 * avg,
                       "launches": n}
    out.update({"frames": len(frames), "iters": T,
                "point_component_evals": evals,
                "speedup": out["plain_ms"] / out["batched_ms"],
                "workload": "64 synthetic depth frames subsampled to "
                            "N_f~U[20000,300000], K_f~U[16,200], k-means++ "
                            "labels, lambda=1e-3"})
    if single_evals_per_s:
        out["batched_vs_single_frame_evals_rate"] = out["batched_evals_per_s"] / single_evals_per_s
    return out


def lidar_fit(T=50, reps=3):
    """The LiDAR-scan fit: N = 2,000,000, K = 1000, T iterations."""
    import torch

    import paper_2307_00071_amd as gmm
    from paper_2307_00071_amd import _lib, synth

    dev = torch.device("cuda:0")
    K = 1000
    X = synth.lidar_scan(0)
    N = X.shape[0]
    pts = torch.from_numpy(X).to(dev)
    lab, _ = gmm.kmeanspp(pts, K, seed=1)
    ws = torch.empty(gmm.fit_workspace_bytes(N, K, T), dtype=torch.uint8, device=dev)
    out = {"workload": "synthetic 64-ring LiDAR scan (elevation -25..+15 deg, "
                       "0.2 deg azimuth, planes and cylinders up to 80 m, "
                       "0.02 m range noise), GPU k-means++ labels (draws from "
                       "seed 1), lambda=1e-3",
           "N": N, "K": K, "iters": T, "tile_shape": _lib.tile_config(N, K)}
    for mode in ("two_pass", "shifted"):
        def fit():
            return gmm.fit(pts, K, iters=T, reg_covar=1e-3, labels=lab,
                           moment_mode=mode, workspace=ws)
        for _ in range(2):
            fit()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fit()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[mode + "_ms"] = 1e3 * dt
        out[mode + "_evals_per_s"] = N * K * T / dt
        out[mode + "_final_loglik"] = float(r.loglik[-1].item())
    _lib.profile_read()
    _lib.profile_pairs()
    _lib.profile_enable(1)
    gmm.fit(pts, K, iters=T, reg_covar=1e-3, labels=lab, workspace=ws)
    torch.cuda.synchronize()
    _lib.profile_enable(0)
    tile_ms, launches = _lib.profile_read()
    pe, pa = _lib.profile_pairs()
    out["tile_avg_launch_us"] = 1e3 * tile_ms / max(launches, 1)
    out["evaluated_pair_fraction"] = pe / max(pa, 1)
    return out


def kinit_bench(reps=3, cpu=True):
    """GPU k-means++ seeding against the oracle's (same draws)."""
    import numpy as np
    import torch

    import paper_2307_00071_amd as gmm
    from paper_2307_00071_amd import synth

    dev = torch.device("cuda:0")
    out = {}
    for name, X, K in (("depth_frame", synth.depth_frame(0), 100),
                       ("lidar_scan", synth.lidar_scan(0), 1000)):
        N = X.shape[0]
        pts = torch.from_numpy(X).to(dev)
        u = np.random.default_rng(1).random(K)
        ws = torch.empty(gmm.kmeanspp_workspace_bytes(N, K), dtype=torch.uint8, device=dev)
        gmm.kmeanspp(pts, K, u=u, workspace=ws)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            lab, cen = gmm.kmeanspp(pts, K, u=u, workspace=ws)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        r = {"N": N, "K": K, "gpu_ms": 1e3 * best}
        if cpu:
            import oracle
            t0 = time.perf_counter()
            rc, rl = oracle.kmeanspp(X.astype(np.float64), K, u)
            r["cpu_baseline"] = {"ms": 1e3 * (time.perf_counter() - t0),
                                 "cores": oracle.get_threads(), "kind": "oracle",
                                 "sample": "the whole seeding, same draws"}
            r["identical_to_oracle"] = bool((cen.cpu().numpy() == rc).all() and
                                            (lab.cpu().numpy() == rl).all())
        out[name] = r
    return out


def blobs_fit(reps=10):
    """The small fit: N = 10,000 points from 8 anisotropic Gaussians (1250
    each), K = 8, T = 50, lambda = 1e-3, seeded by the GPU k-means++ (draws
    from seed 1).  Fits replayed as captured graphs; median of reps."""
    import numpy as np
    import torch

    import oracle
    import paper_2307_00071_amd as gmm
    from paper_2307_00071_amd import synth

    dev = torch.device("cuda:0")
    X, _, _ = synth.gaussian_blobs(0)
    N, K, T = X.shape[0], 8, 50
    pts = torch.from_numpy(X).to(dev)
    lab, _ = gmm.kmeanspp(pts, K, seed=1)
    ws = torch.empty(gmm.fit_workspace_bytes(N, K, T), dtype=torch.uint8, device=dev)

    def fit():
        return gmm.fit(pts, K, iters=T, reg_covar=1e-3, labels=lab, workspace=ws)

    for _ in range(3):
        fit()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = fit()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    labn = lab.cpu().numpy()
    t0 = time.perf_counter()
    Lo = oracle.fit(X, K, 1e-3, T, labels=labn)[3]
    dto = time.perf_counter() - t0
    L = r.loglik.cpu().numpy()
    return {"workload": "N=10000 points from 8 anisotropic Gaussians (means "
                        "U[0,10]^3 m, s~U[0.05,0.5] m), K=8, T=50, lambda=1e-3, "
                        "GPU k-means++ labels (seed 1)",
            "N": N, "K": K, "iters": T, "ms_per_fit": 1e3 * dt,
            "us_per_iteration": 1e6 * dt / T, "em_iters_per_s": T / dt,
            "final_loglik": float(L[-1]),
            "final_loglik_rel_err_vs_oracle": abs(L[-1] - Lo[-1]) / max(abs(Lo[-1]), N),
            "cpu_baseline": {"ms_per_fit": 1e3 * dto, "us_per_iteration": 1e6 * dto / T,
                             "cores": oracle.get_threads(), "kind": "oracle",
                             "sample": "the whole 50-iteration fit from the same labels"}}


def model4d_bench(reps=5, cpu=True):
    """The paper's 4D (x, y, z, intensity) model on the synthetic
    depth-intensity frame: EM fits at the full 640 x 480 frame and at the
    2x-reduced 320 x 240 image (every other pixel), K = 100, T = 100, from
    k-means++ labels of the xyz part; then the conditional intensity at every
    pixel's location and 640 x 480 joint samples (the paper's examples).
    Fits replayed as captured graphs, median of reps; the whole-iteration
    time stands in for the tile kernel in the roofline figure (a lower bound
    of the kernel's rate).  The FP64 4D
    oracle (numpy) is timed on 2 iterations of the 320 x 240 fit."""
    import numpy as np
    import torch

    import paper_2307_00071_amd as gmm
    from paper_2307_00071_amd import synth

    dev = torch.device("cuda:0")
    X = synth.depth_intensity_frame(0)
    out = {"workload": "synthetic depth-intensity frame, 4D EM K=100 T=100 lambda=1e-3 "
                       "from k-means++ labels of xyz; conditional intensity; joint sampling"}
    K, T = 100, 100
    for name, Xs in (("640x480", X), ("320x240", X.reshape(480, 640, 4)[::2, ::2].reshape(-1, 4))):
        Xs = np.ascontiguousarray(Xs)
        N = Xs.shape[0]
        pts = torch.from_numpy(Xs).to(dev)
        lab, _ = gmm.kmeanspp(torch.from_numpy(np.ascontiguousarray(Xs[:, :3])).to(dev), K, seed=1)
        ws = torch.empty(gmm.fit4_workspace_bytes(N, K, T), dtype=torch.uint8, device=dev)
        for _ in range(3):
            r = gmm.fit4(pts, K, iters=T, labels=lab, workspace=ws)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = gmm.fit4(pts, K, iters=T, labels=lab, workspace=ws)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        evals = N * K * T
        ach = FLOP_PER_EVAL_4D * N * K / (dt / T) / 1e12
        sec = {"N": N, "K": K, "iters": T, "ms_per_fit": 1e3 * dt, "evals_per_s": evals / dt,
               "final_loglik": float(r.loglik[-1].item()),
               "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_VECTOR,
                            "unit": "TFLOP/s", "frac": ach / PEAK_FP32_VECTOR,
                            "kernel": "whole EM iteration (4D tile kernel + reduction + update)",
                            "flop_per_eval": FLOP_PER_EVAL_4D}}
        if name == "320x240":
            locs = pts[:, :3].contiguous()
            gmm.color_conditional(locs, r.weights, r.means, r.covariances)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                gmm.color_conditional(locs, r.weights, r.means, r.covariances)
            torch.cuda.synchronize()
            sec["color_conditional_ms"] = 1e3 * (time.perf_counter() - t0) / reps
            rng = np.random.default_rng(2)
            m = 640 * 480
            u = torch.from_numpy(rng.random(m)).to(dev)
            z = torch.from_numpy(rng.standard_normal((m, 4)).astype(np.float32)).to(dev)
            gmm.joint_dist_sample(r.weights, r.means, r.covariances, m, u=u, z=z)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                gmm.joint_dist_sample(r.weights, r.means, r.covariances, m, u=u, z=z)
            torch.cuda.synchronize()
            sec["joint_dist_sample_640x480_ms"] = 1e3 * (time.perf_counter() - t0) / reps
            if cpu:
                from oracle import gmm4 as o4
                labn = lab.cpu().numpy()
                t0 = time.perf_counter()
                o4.fit(Xs.astype(np.float64), K, 1e-3, 2, labels=labn)
                dto = time.perf_counter() - t0
                sec["cpu_baseline"] = {"ms_per_iteration": 1e3 * dto / 3, "cores": 1,
                                       "kind": "oracle",
                                       "sample": "label M-step + 2 EM iterations of the same fit "
                                                 "(numpy FP64), per pass"}
        out[name] = sec
    return out


def pipeline_bench(reps=3):
    """The paper's GPU pipeline end to end on the 320 x 240 depth-intensity
    frame (76,800 4D points): mean shift for K at bandwidth h, k-means++
    seeding of K centres on the xyz part (draws from seed 1), then the 4D EM
    fit (T = 100, lambda = 1e-3) from those labels; bandwidths 0.2 and 0.3,
    the smallest of the synthetic frame whose K fits the 4D fit (K <= 512).
    Median over reps of each stage and of the whole chain."""
    import numpy as np
    import torch

    import paper_2307_00071_amd as gmm
    from paper_2307_00071_amd import synth

    dev = torch.device("cuda:0")
    X = np.ascontiguousarray(
        synth.depth_intensity_frame(0).reshape(480, 640, 4)[::2, ::2].reshape(-1, 4))
    pts = torch.from_numpy(X).to(dev)
    xyz = pts[:, :3].contiguous()
    N, T = X.shape[0], 100
    msws = torch.empty(gmm.meanshift_workspace_bytes(N, 4), dtype=torch.uint8, device=dev)
    out = {"workload": "320x240 depth-intensity frame: mean shift (K) -> k-means++ on xyz "
                       "-> 4D EM, T=100, lambda=1e-3"}
    for h in (0.2, 0.3):
        stages = {"meanshift": [], "kmeanspp": [], "fit4": [], "total": []}
        K = None
        for rep in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = gmm.meanshift(pts, h, workspace=msws)
            K = info["n_modes"]
            t1 = time.perf_counter()
            lab, _ = gmm.kmeanspp(xyz, K, seed=1)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            r = gmm.fit4(pts, K, iters=T, labels=lab)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            if rep == 0:
                continue   # warm-up
            stages["meanshift"].append(t1 - t0)
            stages["kmeanspp"].append(t2 - t1)
            stages["fit4"].append(t3 - t2)
            stages["total"].append(t3 - t0)
        out["h=%g" % h] = {"K": K, "final_loglik": float(r.loglik[-1].item()),
                           **{k + "_ms": 1e3 * float(np.median(v)) for k, v in stages.items()}}
    return out


def meanshift_bench(reps=5, cpu=True, cpu_seeds=60):
    """Component count by mean shift on the 4D depth-intensity frame at the
    paper's 2x-reduced image size (320 x 240 = 76,800 points, every other
    pixel of the synthetic 640 x 480 frame), bandwidths 0.015 (the paper's
    example), 0.03 and 0.1 (larger neighbourhoods, K ~ 2,300); median of
    reps whole calls.  The CPU baseline is the
    FP64 oracle's per-seed mean shift on a seeded sample of the seeds,
    scaled to seeds per second (the merge is not timed there)."""
    import numpy as np
    import torch

    import paper_2307_00071_amd as gmm
    from paper_2307_00071_amd import synth

    dev = torch.device("cuda:0")
    X = np.ascontiguousarray(
        synth.depth_intensity_frame(0).reshape(480, 640, 4)[::2, ::2].reshape(-1, 4))
    pts = torch.from_numpy(X).to(dev)
    ws = torch.empty(gmm.meanshift_workspace_bytes(X.shape[0], 4), dtype=torch.uint8,
                     device=dev)
    out = {"workload": "320x240 depth-intensity frame (N=76800, 4D), flat-kernel mean "
                       "shift over binned seeds, max_iter=300"}
    for h in (0.015, 0.03, 0.1):
        gmm.meanshift(pts, h, workspace=ws)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            _, _, info = gmm.meanshift(pts, h, workspace=ws)
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        r = {"bandwidth": h, "ms": 1e3 * dt, "seeds": info["n_seeds"], "K": info["n_modes"],
             "merge_rounds": info["rounds"], "max_iters": info["max_iters"],
             "seeds_per_s": info["n_seeds"] / dt}
        if cpu:
            from oracle import gbms as og
            X64 = X.astype(np.float64)
            seeds = og.bin_seeds(X64, h)
            pick = np.random.default_rng(3).choice(seeds.shape[0], cpu_seeds, replace=False)
            t0 = time.perf_counter()
            for i in pick:
                og.shift_seed(X64, seeds[i], h, 300)
            dto = time.perf_counter() - t0
            r["cpu_baseline"] = {"seeds_per_s": cpu_seeds / dto,
                                 "est_ms_all_seeds": 1e3 * dto / cpu_seeds * info["n_seeds"],
                                 "cores": 1, "kind": "oracle",
                                 "sample": "%d seeded seeds' mean shift (numpy, "
                                           "brute-force radius queries)" % cpu_seeds}
        out["h=%g" % h] = r
    return out


def d2d_bench(reps=5, cpu=True):
    """D2D registration of two depth-frame mixtures (K = 100 and K = 1000 on
    each side; mixtures fitted on the GPU to two renders of the synthetic
    depth frame, the second moved by a known pose): 10 isoplanar + 30
    anisotropic iterations, median of reps whole calls; the FP64 oracle's
    registration timed beside it (K = 100 whole, K = 1000 one objective +
    gradient evaluation)."""
    import numpy as np
    import torch

    import paper_2307_00071_amd as gmm
    from paper_2307_00071_amd import synth

    dev = torch.device("cuda:0")
    pose = synth.random_pose(5, max_angle=0.15, max_trans=0.2)
    out = {"workload": "source/target mixtures of two renders of the depth frame "
                       "(target moved by |omega| <= 0.15 rad, |t| <= 0.2 m), "
                       "10 isoplanar + 30 anisotropic Gauss-Newton iterations, FP64"}
    for K in (100, 1000):
        mixes = []
        for noise in (None, 77):
            X = synth.depth_frame(0, noise_seed=noise) if noise else synth.depth_frame(0)
            pts = torch.from_numpy(X).to(dev)
            lab, _ = gmm.kmeanspp(pts, K, seed=1)
            r = gmm.fit(pts, K, iters=20, labels=lab)
            mixes.append((r.weights, r.means, r.covariances))
        w, mu, cov = mixes[1]
        import math
        th = float(np.linalg.norm(pose[:3]))
        k = pose[:3] / th
        Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        R = np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * Kx @ Kx
        Rt = torch.as_tensor(R, dtype=torch.float32, device=dev)
        tt = torch.as_tensor(pose[3:], dtype=torch.float32, device=dev)
        tgt = (w, mu @ Rt.T + tt, Rt @ cov @ Rt.T)
        src = mixes[0]
        gmm.d2d_register(src, tgt, iters_iso=10, iters_aniso=30)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            T, hist, counts = gmm.d2d_register(src, tgt, iters_iso=10, iters_aniso=30)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        Tn = T.cpu().numpy()
        cn = counts.cpu().numpy()
        it = int(cn.sum())
        # FP64 work: a value-pass pair term ~45 FLOP (+ log, exp), a
        # statistics-pass pair term ~290 FLOP (+ log, exp); per iteration one
        # statistics pass and eight value passes, per stage one value pass
        flop = K * K * (it * (D2D_FLOP_STATS + 8 * D2D_FLOP_VALUE) + 2 * D2D_FLOP_VALUE)
        r = {"K": K, "ms": 1e3 * dt, "iterations": [int(x) for x in cn],
             "pairs_per_iteration": K * K * 9,
             "pair_evals_per_s": K * K * (9 * it + 2) / dt,
             "roofline": {"bound": "fp64 alu", "achieved": flop / dt / 1e12,
                          "peak": PEAK_FP64_VECTOR, "unit": "TFLOP/s",
                          "frac": flop / dt / 1e12 / PEAK_FP64_VECTOR,
                          "kernel": "whole registration (all its launches)"},
             "rot_err_rad": float(np.linalg.norm(Tn[:3, :3] - R)),
             "trans_err_m": float(np.linalg.norm(Tn[:3, 3] - pose[3:]))}
        if cpu:
            from oracle import d2d as od
            s64 = tuple(a.cpu().numpy().astype(np.float64) for a in src)
            t64 = tuple(a.cpu().numpy().astype(np.float64) for a in tgt)
            t0 = time.perf_counter()
            if K <= 100:
                od.register(np.eye(4), s64, t64, iters_iso=10, iters_aniso=30)
                what = "the whole registration"
            else:
                od.objective_grad(np.zeros(6), s64, t64)
                what = "one objective + gradient evaluation (1e6 pairs)"
            r["cpu_baseline"] = {"ms": 1e3 * (time.perf_counter() - t0), "cores": 1,
                                 "kind": "oracle", "sample": what}
        out["K=%d" % K] = r
    return out


def registration(reps=20, cpu=True):
    """Registration likelihood and gradient: a K = 200 mixture fitted (GPU,
    20 iterations from k-means++ labels) to the depth frame, a source of
    N = 100,000 points from a second noisy render of the scene under a
    random pose (|omega| <= 0.3 rad, |t| <= 0.5 m)."""
    import numpy as np
    import torch

    import oracle
    import paper_2307_00071_amd as gmm
    from paper_2307_00071_amd import _lib, synth

    dev = torch.device("cuda:0")
    K, Nsrc = 200, 100_000
    Xt = torch.from_numpy(synth.depth_frame(0)).to(dev)
    lab, _ = gmm.kmeanspp(Xt, K, seed=1)
    th = gmm.fit(Xt, K, iters=20, reg_covar=1e-3, labels=lab)
    w, mu, cov = th.weights, th.means, th.covariances
    Y = synth.depth_frame(0, noise_seed=7)
    rng = np.random.default_rng(101)
    src = np.ascontiguousarray(Y[np.sort(rng.choice(Y.shape[0], Nsrc, replace=False))])
    pose = torch.from_numpy(synth.random_pose(2).astype(np.float32)).to(dev)
    pts = torch.from_numpy(src).to(dev)

    def fwd():
        return gmm.loglik(pts, w, mu, cov, pose6=pose, check=False)

    def bwd():
        return gmm.loglik_backward(pts, w, mu, cov, pose6=pose, check=False)

    def both():
        p = pose.clone().requires_grad_(True)
        x = pts.clone().requires_grad_(True)
        tw, tm, tc = (a.clone().requires_grad_(True) for a in (w, mu, cov))
        L = gmm.GMMLogLik.apply(x, p, tw, tm, tc)
        L.backward()
        return L

    out = {"workload": "K=200 mixture fitted to the 640x480 depth frame; "
                       "N=100000 source points from a second noisy render "
                       "under a random SE(3) pose (|omega|<=0.3 rad, "
                       "|t|<=0.5 m); gradient w.r.t. pose, points, weights, "
                       "means, covariances",
           "N": Nsrc, "K": K}
    for name, fn in (("forward", fwd), ("backward", bwd), ("forward_backward_autograd", both)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        out[name + "_ms"] = 1e3 * float(np.median(times))
    out["evals_per_s"] = Nsrc * K / (out["forward_backward_autograd_ms"] * 1e-3)
    # kernel times: each timed pair covers PROFILE_REPS back-to-back launches
    kern = {}
    for name, fn, flop in (("forward", fwd, FLOP_PER_EVAL_FWD),
                           ("backward", bwd, FLOP_PER_EVAL_BWD)):
        _lib.profile_read()
        _lib.profile_pairs()
        _lib.profile_enable(PROFILE_REPS)
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        _lib.profile_enable(0)
        ms, n = _lib.profile_read()
        pe, pa = _lib.profile_pairs()
        avg = ms / max(n, 1) * 1e-3
        ach = flop * Nsrc * K / avg / 1e12
        kern[name] = {"avg_launch_us": 1e6 * avg, "launches": n,
                      "achieved": ach, "frac": ach / PEAK_FP32_VECTOR,
                      "evaluated_pair_fraction": pe / max(pa, 1),
                      "flop_per_eval": flop}
    out["kernels"] = kern
    out["roofline"] = {"bound": "alu", "kernel": "em_bwd_kernel (dense)",
                       "achieved": kern["backward"]["achieved"],
                       "peak": PEAK_FP32_VECTOR, "unit": "TFLOP/s",
                       "frac": kern["backward"]["frac"], "traffic": None}
    if cpu:
        th64 = tuple(a.cpu().numpy().astype(np.float64) for a in (w, mu, cov))
        p64 = pose.cpu().numpy().astype(np.float64)
        oracle.loglik_pose(src, p64, *th64)
        t0 = time.perf_counter()
        for _ in range(3):
            oracle.loglik_pose(src, p64, *th64)
            oracle.loglik_grad(src, p64, *th64)
        dto = (time.perf_counter() - t0) / 3
        out["cpu_baseline"] = {"value": Nsrc * K / dto, "unit": "point-component evals/s",
                               "ms": 1e3 * dto, "cores": oracle.get_threads(),
                               "kind": "oracle",
                               "sample": "likelihood + analytic gradient of the same "
                                         "problem, FP64, mean of 3"}
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; the fit of one frame runs "
              "on a single MI355X (sharding over several GPUs is not "
              "implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2307_00071_amd as gmm
    from paper_2307_00071_amd import _lib, synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    K, T = args.k, args.iters
    X = synth.depth_frame(0)
    lab = synth.kmeanspp_labels(X, K, 1)
    N = X.shape[0]
    pts = torch.from_numpy(X).to(dev)
    labt = torch.from_numpy(lab).to(dev)
    ws = torch.empty(gmm.fit_workspace_bytes(N, K, T), dtype=torch.uint8,
                     device=dev)

    def step():
        return gmm.fit(pts, K, iters=T, reg_covar=1e-3, labels=labt,
                       workspace=ws)

    for _ in range(max(args.warmup, 2)):   # the second call captures the graph
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # second timed region: the same fits, direct launches, kernel events
    _lib.profile_read()
    _lib.profile_enable(PROFILE_REPS)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    _lib.profile_enable(0)
    tile_ms, launches = _lib.profile_read()
    pairs_eval, pairs_all = _lib.profile_pairs()
    shape = _lib.tile_config(N, K)
    L = r.loglik.cpu().numpy()
    assert np.all(np.isfinite(L)), "non-finite log-likelihood"

    ms_per_step = 1e3 * dt / args.steps
    evals = N * K * T
    value = evals / (dt / args.steps)
    avg_s = tile_ms / max(launches, 1) * 1e-3
    achieved = FLOP_PER_EVAL * N * K / avg_s / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "point-component evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single-frame EM fit, synthetic 640x480 depth "
                               "frame N=%d, K=%d, T=%d iterations, k-means++ "
                               "labels, lambda=1e-3, shifted moments" % (N, K, T),
                   "N": N, "K": K, "iters": T},
        "em_iters_per_s": T / (dt / args.steps),
        "final_loglik": float(L[-1]),
        "roofline": {"bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_VECTOR, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR,
                     "traffic": tile_traffic_bytes(N, K),
                     "kernel": "%s (E-step + M-step statistics), shape %s"
                               % ("em_cull_kernel" if shape.startswith("c")
                                  else "em_tile_kernel", shape),
                     "avg_launch_us": avg_s * 1e6, "launches": launches,
                     "peak_nonpacked": PEAK_FP32_NONPACKED,
                     "frac_nonpacked": achieved / PEAK_FP32_NONPACKED,
                     # share of the N*K point-component pairs the kernel
                     # computed (the rest were shown to be exactly zero)
                     "evaluated_pair_fraction": pairs_eval / max(pairs_all, 1),
                     # the same time against the FLOPs of the pairs the
                     # kernel actually evaluated (dense-equivalent above)
                     "achieved_on_evaluated_pairs":
                         achieved * pairs_eval / max(pairs_all, 1),
                     "frac_on_evaluated_pairs":
                         achieved * pairs_eval / max(pairs_all, 1) / PEAK_FP32_VECTOR},
    }
    cpu = not args.no_cpu_baseline
    sections = [
        ("batched", not args.no_batched,
         lambda: batched_vs_plain(args.batched_iters, single_evals_per_s=value)),
        ("lidar", not args.no_lidar, lidar_fit),
        ("kinit", not args.no_kinit, lambda: kinit_bench(cpu=cpu)),
        ("blobs", not args.no_blobs, blobs_fit),
        ("registration", not args.no_registration, lambda: registration(cpu=cpu)),
        ("model4d", not args.no_model4d, lambda: model4d_bench(cpu=cpu)),
        ("meanshift", not args.no_meanshift, lambda: meanshift_bench(cpu=cpu)),
        ("pipeline", not args.no_pipeline, pipeline_bench),
        ("d2d", not args.no_d2d, lambda: d2d_bench(cpu=cpu)),
    ]
    for name, on, run in sections:
        if on:
            out[name] = run()
            print("bench.py: %s done" % name, file=sys.stderr, flush=True)
    if cpu:
        out["cpu_baseline"] = cpu_baseline(X, lab, K, T, args.cpu_seconds)
        out["cpu_baseline_1thread"] = cpu_baseline(X, lab, K, T, 4.0, threads=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
