// Device code of the MI355X (gfx950) GMM EM library: helpers and kernels.
// Included once, by gmm.hip.
//
// One EM iteration is three launches:
//   tile loop  - persistent tiles of T points.  E-phase: lanes = points,
//                components wave-uniform (scalar loads of the parameter
//                block), e_pb = 2^(log2(e) (l_pb - C)) into LDS and the
//                per-point normaliser (eq. 1-3).  M-phase: lanes =
//                (component, point subset); each lane reads gamma_pb from LDS
//                and keeps its own sum g, sum g d, sum g d d^T in registers
//                (FP32 over a tile, FP64 across tiles): no cross-lane
//                reduction per point.  One FP64 partial row per block.
//   reduce_rows_kernel, update_kernel - fixed-order FP64 sum of the rows
//                (wide, then one block), and the FP64 M-step, the FP64 3x3
//                Cholesky and the eq. 3 terms for the next iteration.
// Every reduction has a fixed order, so a fit is bitwise reproducible for a
// given launch configuration.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "gmm.h"
#include "wave_f64.hpp"

namespace gmm_dev {

using namespace gmm_wave;

// ------------------------------------------------------------------ constants

constexpr double kLog2e = 1.44269504088896340736;
constexpr double kLn2 = 0.693147180559945309417;
constexpr double kLn2Pi = 1.83787706640934548356;
constexpr double kEpsN = 10.0 * 2.220446049250313080847e-16;  // N_b guard
constexpr int kParStride = 16;   // floats per component in the E-step block
constexpr int kTh64Stride = 16;  // doubles per component in the FP64 state
constexpr int kNStat = 10;       // N, S1 (3), S2 lower triangle (6)

// status bits (device status word)
constexpr uint32_t kStBadArg = 1u << GMM_ERR_INVALID_ARG;
constexpr uint32_t kStNotSpd = 1u << GMM_ERR_NOT_SPD;
constexpr uint32_t kStNonFinite = 1u << GMM_ERR_NONFINITE;

enum TileMode { kSoftStats = 0, kSoftLogLik = 1, kLabels = 2 };
// kUpdNone: only the log-likelihood (and optional FP32 outputs);
// kUpdMeanOnly: the new means become the next pass's shift, the E-step
// block is carried over unchanged; kUpdFull: the complete M-step.
enum UpdMode { kUpdFull = 0, kUpdMeanOnly = 1, kUpdNone = 2 };

// ------------------------------------------------------------------ layout
// E-step parameter block ("cpar"), per component (16 floats):
//   [0..2] mu  [3] (c_b - C) * log2(e)  [4..9] s * P (P00 P10 P11 P20 P21 P22)
//   [10] an upper bound of the Frobenius norm of s * P (tile culling)
// with s = sqrt(log2(e) / 2), c_b = ln pi_b - 3/2 ln 2pi + sum_j ln P_jj
// (eq. 3) and a reference C, so [3] - |P' (x - mu)|^2 = log2(e)(l_nb - C).
// After the K blocks: C * log2(e) as a double.  C is max_b c_b for caller
// parameters and for lambda = 0 (then [3] <= 0), and the static
// 3/2 ln(1 / lambda) - 3/2 ln 2pi - ln K for parameters from an M-step with
// lambda > 0: every eigenvalue of such a Sigma_b is at least lambda, so
// prod_j P_jj <= lambda^-3/2, and pi_b <= 1, hence [3] <= log2 K (a point's
// sum of 2^[3] terms stays below K^2, far from FP32 overflow) while a
// typical weight 1/K keeps [3] near 0, where its float32 rounding is small.
// Shift array: the FP32 point the M-phase subtracts, per component.
// FP64 state ("th64"), per component (16 doubles):
//   [0] pi  [1..3] mu  [4..9] Sigma lower (00 10 11 20 21 22)  [10] N_b

// ------------------------------------------------------- device helpers

__device__ inline void set_status(uint32_t *st, uint32_t bits) {
  atomicOr(st, bits);
}

// Cholesky of the 3x3 SPD matrix with lower triangle C = (00 10 11 20 21 22).
// Returns false on a non-positive or non-finite pivot.
__device__ inline bool chol3(const double *C, double *L) {
  double a = C[0];
  if (!(a > 0.0) || !isfinite(a)) return false;
  double l00 = sqrt(a);
  double l10 = C[1] / l00;
  double b = C[2] - l10 * l10;
  if (!(b > 0.0) || !isfinite(b)) return false;
  double l11 = sqrt(b);
  double l20 = C[3] / l00;
  double l21 = (C[4] - l20 * l10) / l11;
  double c = C[5] - l20 * l20 - l21 * l21;
  if (!(c > 0.0) || !isfinite(c)) return false;
  double l22 = sqrt(c);
  L[0] = l00; L[1] = l10; L[2] = l11; L[3] = l20; L[4] = l21; L[5] = l22;
  return true;
}

// P = L^-1 (lower) by forward substitution, same packed order.
__device__ inline void tri_inv3(const double *L, double *P) {
  double p00 = 1.0 / L[0], p11 = 1.0 / L[2], p22 = 1.0 / L[5];
  double p10 = -L[1] * p00 * p11;
  double p21 = -L[4] * p11 * p22;
  double p20 = -(L[3] * p00 + L[4] * p10) * p22;
  P[0] = p00; P[1] = p10; P[2] = p11; P[3] = p20; P[4] = p21; P[5] = p22;
}

// Cholesky of the SPD 3x3 C and P = L^-1 together: the three diagonal
// reciprocals serve both (3 square roots, 3 divisions).  Returns false on a
// non-positive or non-finite pivot.
__device__ __forceinline__ bool chol_inv3(const double *C, double *P) {
  double a = C[0];
  if (!(a > 0.0) || !isfinite(a)) return false;
  const double l00 = sqrt(a), r0 = 1.0 / l00;
  const double l10 = C[1] * r0, l20 = C[3] * r0;
  const double b = C[2] - l10 * l10;
  if (!(b > 0.0) || !isfinite(b)) return false;
  const double l11 = sqrt(b), r1 = 1.0 / l11;
  const double l21 = (C[4] - l20 * l10) * r1;
  const double c = C[5] - l20 * l20 - l21 * l21;
  if (!(c > 0.0) || !isfinite(c)) return false;
  const double r2 = 1.0 / sqrt(c);
  const double p10 = -l10 * r0 * r1;
  P[0] = r0; P[1] = p10; P[2] = r1;
  P[3] = -(l20 * r0 + l21 * p10) * r2; P[4] = -l21 * r1 * r2; P[5] = r2;
  return true;
}

// The E-step block of one component (all but [3]) from mu and P.
__device__ __forceinline__ void store_eblock(float *q, const double *mu, const double *P) {
  const double s = sqrt(0.5 * kLog2e);
  double fro = 0.0;
  q[0] = (float)mu[0]; q[1] = (float)mu[1]; q[2] = (float)mu[2];
  for (int j = 0; j < 6; ++j) {
    q[4 + j] = (float)(s * P[j]);
    fro += P[j] * P[j];
  }
  // |P'|_F rounded up: the tile-culling bound needs an upper bound of |P'|_2
  q[10] = (float)(s * sqrt(fro) * (1.0 + 1e-6));
}

// Stores one component (pi, mu, Sigma) in the FP64 state, its E-step block
// (all but [3]) and its shift; returns c_b * log2(e), or -inf when Sigma is
// not SPD (the component then contributes 2^-inf = 0 everywhere).
__device__ inline double component_terms(int b, double pi, const double *mu,
                                         const double *C, double Nb,
                                         float *cpar, float4 *shift,
                                         double *th64) {
  double *t = th64 + (size_t)b * kTh64Stride;
  t[0] = pi;
  for (int j = 0; j < 3; ++j) t[1 + j] = mu[j];
  for (int j = 0; j < 6; ++j) t[4 + j] = C[j];
  t[10] = Nb;
  const float mf0 = (float)mu[0], mf1 = (float)mu[1], mf2 = (float)mu[2];
  shift[b] = make_float4(mf0, mf1, mf2, 0.0f);
  float *q = cpar + (size_t)b * kParStride;
  q[0] = mf0; q[1] = mf1; q[2] = mf2;
  double P[6];
  if (!chol_inv3(C, P)) {
    for (int j = 0; j < 6; ++j) q[4 + j] = 0.0f;
    q[10] = 0.0f;
    return -INFINITY;
  }
  store_eblock(q, mu, P);
  // ln pi + sum_j ln P_jj = ln(pi P00 P11 P22), one logarithm
  const double c = log(pi * P[0] * P[2] * P[5]) - 1.5 * kLn2Pi;
  return c * kLog2e;
}

// Block-wide (NT threads) fixed-order tree reductions over NT doubles.
template <int NT>
__device__ inline double block_sum(double v, double *scratch) {
  const int tid = threadIdx.x;
  __syncthreads();
  scratch[tid] = v;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (tid < h) scratch[tid] += scratch[tid + h];
    __syncthreads();
  }
  return scratch[0];
}

template <int NT>
__device__ inline double block_max(double v, double *scratch) {
  const int tid = threadIdx.x;
  __syncthreads();
  scratch[tid] = v;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (tid < h) scratch[tid] = fmax(scratch[tid], scratch[tid + h]);
    __syncthreads();
  }
  return scratch[0];
}

// With sC[b] = c_b * log2(e) for every component: C = max_b c_b, each
// component's [3] = c_b - C and the header C.
template <int NT>
__device__ inline void apply_bound(int K, const double *sC, float *cpar,
                                   double *scratch) {
  double m = -INFINITY;
  for (int b = threadIdx.x; b < K; b += NT) m = fmax(m, sC[b]);
  double C = block_max<NT>(m, scratch);
  if (!isfinite(C)) C = 0.0;
  for (int b = threadIdx.x; b < K; b += NT) {
    const double c = sC[b];
    cpar[(size_t)b * kParStride + 3] = isfinite(c) ? (float)(c - C) : -INFINITY;
  }
  if (threadIdx.x == 0) *reinterpret_cast<double *>(cpar + (size_t)K * kParStride) = C;
}

// Block-wide reductions in a fixed order with two barriers: a DPP wave sum in
// each wave, then the wave results added in wave order by one thread.
template <int NT>
__device__ inline double block_sum_fast(double v, double *scratch) {
  v = wave_sum_f64(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = scratch[0];
    for (int j = 1; j < NT / 64; ++j) t += scratch[j];
    scratch[NT / 64] = t;
  }
  __syncthreads();
  return scratch[NT / 64];
}

template <int NT>
__device__ inline double block_max_fast(double v, double *scratch) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = scratch[0];
    for (int j = 1; j < NT / 64; ++j) t = fmax(t, scratch[j]);
    scratch[NT / 64] = t;
  }
  __syncthreads();
  return scratch[NT / 64];
}

// ------------------------------------------------------------------ M-step
// From the reduced statistics tot[] (column s*K + b: N0, S1 (3), S2 (6); the
// log-likelihood at 10 K) and the shift m the tile kernel subtracted:
//   N_b = N0 + eps,  mu = (S1 + N0 m) / N_b,  delta = mu - m,
//   Sigma = (S2 - S1 delta^T - delta S1^T + N0 delta delta^T) / N_b + lambda I
// which is sum g (x - mu)(x - mu)^T / N_b + lambda I exactly;
//   pi_b = N_b / sum_a N_a, then the eq. 3 terms for the next E-step.
// One block of NT >= K threads, thread b owns component b (registers only);
// scratch holds 2 NT / 64 doubles.  ROW16 (K <= 16: every component in the
// first DPP row): sum N_b and max cb by a row reduction, no scratch and no
// barrier.
template <int NT, bool ROW16 = false>
__device__ __forceinline__ void em_update_block(const double *tot, int K, int umode, double reg,
                                const float *cpar_in, const float4 *shift_in,
                                float *cpar_out, float4 *shift_out,
                                double *th64, double *scratch, uint32_t *status) {
  const int b = threadIdx.x;
  const bool act = b < K;
  if (umode == kUpdMeanOnly) {
    if (act) {
      const double N0 = tot[b];
      const float4 mf = shift_in[b];
      const double Nb = N0 + kEpsN;
      const double m[3] = {mf.x, mf.y, mf.z};
      float mu[3];
      bool fin = isfinite(N0);
      for (int j = 0; j < 3; ++j) {
        const double S1 = tot[(1 + j) * K + b];
        fin = fin && isfinite(S1);
        mu[j] = (float)((S1 + N0 * m[j]) / Nb);
      }
      if (!fin) set_status(status, kStNonFinite);
      shift_out[b] = make_float4(mu[0], mu[1], mu[2], 0.0f);
    }
    // the E-step block of the current parameters carries over
    const int nf = (K + 1) * kParStride;
    for (int i = b; i < nf; i += NT) cpar_out[i] = cpar_in[i];
    return;
  }
  // umode == kUpdFull
  const int ij[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
  double Nb = 0.0, mu[3] = {0.0, 0.0, 0.0}, C[6] = {0, 0, 0, 0, 0, 0};
  if (act) {
    const double N0 = tot[b];
    const double S1[3] = {tot[1 * K + b], tot[2 * K + b], tot[3 * K + b]};
    const float4 mf = shift_in[b];
    const double m[3] = {mf.x, mf.y, mf.z};
    Nb = N0 + kEpsN;
    const double rN = 1.0 / Nb;
    double dl[3];
    for (int j = 0; j < 3; ++j) {
      mu[j] = (S1[j] + N0 * m[j]) * rN;
      dl[j] = mu[j] - m[j];
    }
    bool fin = isfinite(N0) && isfinite(S1[0]) && isfinite(S1[1]) && isfinite(S1[2]);
    for (int j = 0; j < 6; ++j) {
      const int r = ij[j][0], c = ij[j][1];
      const double s2 = tot[(4 + j) * K + b];
      const double v = s2 - S1[r] * dl[c] - dl[r] * S1[c] + N0 * dl[r] * dl[c];
      C[j] = v * rN + ((r == c) ? reg : 0.0);
      fin = fin && isfinite(s2);
    }
    if (!fin) set_status(status, kStNonFinite);
  }
  // Cholesky, P and cb = ln(N_b P00 P11 P22) before any reduction: with
  // pi_b = N_b / N, c_b = cb - ln N - 3/2 ln 2pi, so c_b - max_a c_a =
  // cb - max_a cb_a and one combined reduction (sum N_b, max cb) suffices.
  double P[6] = {0, 0, 0, 0, 0, 0};
  double cb = -INFINITY;
  if (act && chol_inv3(C, P)) cb = log(Nb * P[0] * P[2] * P[5]);
  if (act && !isfinite(cb)) set_status(status, kStNotSpd);
  double sN = act ? Nb : 0.0, mC = cb;
  double Ntot, Mx;
  if constexpr (ROW16) {
    Ntot = row16_sum(sN);
    Mx = row16_max(mC);
  } else {
    for (int off = 32; off > 0; off >>= 1) {
      sN += __shfl_xor(sN, off, 64);
      mC = fmax(mC, __shfl_xor(mC, off, 64));
    }
    constexpr int NWV = NT / 64;
    if ((b & 63) == 0) {
      scratch[b >> 6] = sN;
      scratch[NWV + (b >> 6)] = mC;
    }
    __syncthreads();
    Ntot = scratch[0];
    Mx = scratch[NWV];
#pragma unroll
    for (int j = 1; j < NWV; ++j) {
      Ntot += scratch[j];
      Mx = fmax(Mx, scratch[NWV + j]);
    }
  }
  if (act) {
    double *t = th64 + (size_t)b * kTh64Stride;
    t[0] = Nb / Ntot;
    for (int j = 0; j < 3; ++j) t[1 + j] = mu[j];
    for (int j = 0; j < 6; ++j) t[4 + j] = C[j];
    t[10] = Nb;
    shift_out[b] = make_float4((float)mu[0], (float)mu[1], (float)mu[2], 0.0f);
    float *q = cpar_out + (size_t)b * kParStride;
    if (isfinite(cb)) {
      store_eblock(q, mu, P);
      q[3] = (float)((cb - Mx) * kLog2e);
    } else {
      q[0] = (float)mu[0]; q[1] = (float)mu[1]; q[2] = (float)mu[2];
      for (int j = 0; j < 6; ++j) q[4 + j] = 0.0f;
      q[10] = 0.0f;
      q[3] = -INFINITY;
    }
  }
  if (b == 0) {
    const double Cmax = isfinite(Mx) ? (Mx - log(Ntot) - 1.5 * kLn2Pi) * kLog2e : 0.0;
    *reinterpret_cast<double *>(cpar_out + (size_t)K * kParStride) = Cmax;
  }
}

// Caller-supplied theta_0 (FP32 w, mu, cov) -> FP64 state and E-step block;
// weights used as given.  One block of kPreThreads threads.
constexpr int kPreThreads = 1024;
__global__ __launch_bounds__(kPreThreads) void precompute_kernel(
    const float *__restrict__ w, const float *__restrict__ mu,
    const float *__restrict__ cov, int K, float *cpar, float4 *shift,
    double *th64, uint32_t *status) {
  __shared__ double scratch[kPreThreads];
  __shared__ double sC[GMM_MAX_K];
  for (int b = threadIdx.x; b < K; b += kPreThreads) {
    double pi = w[b];
    double m[3] = {mu[3 * b], mu[3 * b + 1], mu[3 * b + 2]};
    const float *c = cov + 9 * b;
    double C[6] = {c[0], c[3], c[4], c[6], c[7], c[8]};
    if (!(pi > 0.0) || !isfinite(pi) || !isfinite(m[0]) || !isfinite(m[1]) ||
        !isfinite(m[2])) {
      set_status(status, kStBadArg);
      pi = 1.0;
    }
    const double cc = component_terms(b, pi, m, C, 0.0, cpar, shift, th64);
    if (!isfinite(cc)) set_status(status, kStNotSpd);
    sC[b] = cc;
  }
  apply_bound<kPreThreads>(K, sC, cpar, scratch);
}

// ------------------------------------------------------------ stage kernel
// AoS N x 3 (caller) -> float4 (x, y, z, tag) padded to a tile multiple.
// tag (int bits) = label in label mode, 0 for a real point otherwise, and -1
// for padding.  With a pose, y = R x + t in FP32.
__global__ void stage_kernel(const float *__restrict__ pts, int64_t n,
                             int64_t npad, const int32_t *__restrict__ labels,
                             int K, const float *__restrict__ Rt,
                             float4 *__restrict__ out, uint32_t *status) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  if (i >= n) {
    out[i] = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
    return;
  }
  float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
    set_status(status, kStNonFinite);
    x = y = z = 0.0f;
  }
  if (Rt) {
    float u = fmaf(Rt[0], x, fmaf(Rt[1], y, fmaf(Rt[2], z, Rt[9])));
    float v = fmaf(Rt[3], x, fmaf(Rt[4], y, fmaf(Rt[5], z, Rt[10])));
    float w = fmaf(Rt[6], x, fmaf(Rt[7], y, fmaf(Rt[8], z, Rt[11])));
    x = u; y = v; z = w;
  }
  int tag = 0;
  if (labels) {
    tag = labels[i];
    if (tag < 0 || tag >= K) {
      set_status(status, kStBadArg);
      tag = -1;
    }
  }
  out[i] = make_float4(x, y, z, __int_as_float(tag));
}

// --------------------------------------------------------------- pose kernel
// R = exp([omega]_x) (Rodrigues), the SO(3) left Jacobian J, both FP64, and
// an FP32 copy (R row-major, t) for the staging kernel.
// pose64: [0..8] R, [9..11] t, [12..20] J.
__global__ void pose_kernel(const float *__restrict__ pose6, double *pose64,
                            float *Rt32) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double w[3] = {pose6[0], pose6[1], pose6[2]};
  double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double th = sqrt(th2), a, bb, e;
  if (th < 1e-4) {
    a = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    bb = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    e = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    a = sin(th) / th;
    bb = (1.0 - cos(th)) / th2;
    e = (th - sin(th)) / (th2 * th);
  }
  double S[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  double S2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += S[i * 3 + k] * S[k * 3 + j];
      S2[i * 3 + j] = s;
    }
  for (int i = 0; i < 9; ++i) {
    double id = (i % 4 == 0) ? 1.0 : 0.0;
    pose64[i] = id + a * S[i] + bb * S2[i];        // R
    pose64[12 + i] = id + bb * S[i] + e * S2[i];   // J_l
    Rt32[i] = (float)pose64[i];
  }
  for (int j = 0; j < 3; ++j) {
    pose64[9 + j] = pose6[3 + j];
    Rt32[9 + j] = pose6[3 + j];
  }
}

// Clears the status word and the ticket counters and, for a label start,
// the shift array (the first label pass accumulates about the origin).
__global__ void init_kernel(uint32_t *status, unsigned *counters, int ncnt,
                            float4 *shift, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  if (i == 0) *status = 0u;
  for (int j = i; j < ncnt; j += stride) counters[j] = 0u;
  if (shift)
    for (int b = i; b < K; b += stride) shift[b] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// ------------------------------------------------------------ tile kernel
//
// Per tile of T points (T = one wave of points):
//  E-phase, lanes = (point p, component group g): each lane walks its
//  group's components (wave-uniform, scalar loads) and forms
//    l'_pb = log2(e) (l_pb - C),  C = max_a c_a  (so l'_pb <= 0),
//  e_pb = 2^l'_pb.  The per-point sum s_p = sum_b e_pb then gives
//  lse_p = ln 2 (C' + log2 s_p) and gamma_pb = e_pb / s_p.  When s_p falls
//  below 2^-100 (a point far from every component) the point is redone
//  exactly with its own maximum, so nothing underflows.
//  M-phase, lanes = (component b, point subset q): a lane reads gamma_pb for
//  its TRIP consecutive points from LDS and accumulates
//    N += g, S1 += g d, S2 += g d d^T,  d = x_p - m_b  (FP32 over the tile,
//  then FP64), m_b the shift array.
// With NCH > 1 (large K) the LDS holds one chunk of components at a time:
// the E-phase first forms s_p only, then each chunk recomputes its e_pb.

template <int BLOCK, int T>
struct TileShape {
  static constexpr int G = BLOCK / T;  // component groups in the E-phase
  // LDS row: T points + zero pad (odd stride: conflict-free), long enough
  // for every point-subset split the host may pick (P * TRIP <= TS)
  static constexpr int TS = T + (T == 64 ? 1 : 3);
  static_assert(BLOCK % T == 0, "tile must divide the block");
  static_assert(T % 64 == 0, "a wave must hold one component group");
};

// LDS: [E (also the end-of-kernel subset sums)][Xs][reds][Mp][wL]
template <int BLOCK, int T>
__host__ __device__ constexpr size_t tile_lds_bytes_e(int K, int KC) {
  size_t e = (size_t)KC * TileShape<BLOCK, T>::TS * sizeof(float);
  (void)K;
  size_t d = (size_t)BLOCK * sizeof(double);
  size_t m = e > d ? e : d;
  return (m + 15) & ~(size_t)15;
}

template <int BLOCK, int T>
__host__ __device__ constexpr size_t tile_lds_bytes(int K, int KC) {
  using S = TileShape<BLOCK, T>;
  return tile_lds_bytes_e<BLOCK, T>(K, KC) + S::TS * sizeof(float4) +
         (size_t)S::G * T * sizeof(float) + T * sizeof(float) +
         (BLOCK / 64) * sizeof(double);
}

// Zero the pad columns [T, TS) of the first rows E rows and the pad
// entries of Xs: the last point subset reads them with weight 0.
template <int TS, int T, int BLOCK>
__device__ __forceinline__ void zero_pad(float *E, float4 *Xs, int rows) {
  constexpr int W = TS - T;
  for (int i = threadIdx.x; i < rows * W; i += BLOCK) E[(i / W) * TS + T + i % W] = 0.0f;
  if (threadIdx.x < W) Xs[T + threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// l'_pb of one component (eq. 3 in log2 units, relative to the bound).
__device__ __forceinline__ float comp_logterm(const float *__restrict__ q,
                                              float x, float y, float z) {
  float d0 = x - q[0], d1 = y - q[1], d2 = z - q[2];
  float z0 = q[4] * d0;
  float z1 = fmaf(q[5], d0, q[6] * d1);
  float z2 = fmaf(q[7], d0, fmaf(q[8], d1, q[9] * d2));
  float l = fmaf(-z0, z0, q[3]);
  l = fmaf(-z1, z1, l);
  return fmaf(-z2, z2, l);
}

// Sufficient statistics of one component over TRIP consecutive points.
template <int TRIP>
__device__ __forceinline__ void mstep_run(const float *Eb, const float4 *Xb,
                                          float4 sh, double *acc) {
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f, a5 = 0.f, a6 = 0.f,
        a7 = 0.f, a8 = 0.f, a9 = 0.f;
#pragma unroll
  for (int j = 0; j < TRIP; ++j) {
    const float4 xr = Xb[j];
    const float gm = Eb[j] * xr.w;
    const float d0 = xr.x - sh.x, d1 = xr.y - sh.y, d2 = xr.z - sh.z;
    const float w0 = gm * d0, w1 = gm * d1, w2 = gm * d2;
    a0 += gm;
    a1 += w0; a2 += w1; a3 += w2;
    a4 = fmaf(w0, d0, a4);
    a5 = fmaf(w1, d0, a5);
    a6 = fmaf(w1, d1, a6);
    a7 = fmaf(w2, d0, a7);
    a8 = fmaf(w2, d1, a8);
    a9 = fmaf(w2, d2, a9);
  }
  acc[0] += a0; acc[1] += a1; acc[2] += a2; acc[3] += a3; acc[4] += a4;
  acc[5] += a5; acc[6] += a6; acc[7] += a7; acc[8] += a8; acc[9] += a9;
}

// Integer arguments of the tile kernel (pointers are separate __restrict__
// arguments so the parameter block is read with scalar loads).
struct TileArgs {
  int ntiles, K, KC, P, mode, ncols;
  // kernel timing only: the culled kernel adds the (tile, component) pairs
  // it evaluated here; NULL otherwise
  unsigned long long *pairs = nullptr;
  // fits with a tolerance: bit 0 set = converged, the pass does nothing
  const unsigned *conv = nullptr;
  // order of a partial row: 0 = statistic-major (statistic j of component
  // b at j K + b); 1 = component-major (at b kNStat + j: a component's ten
  // sums adjacent), read by the fused reduction + M-step.  The
  // log-likelihood sum is last either way.
  int cmaj = 0;
};

#ifndef GMM_TILE_WPE
#define GMM_TILE_WPE 1
#endif
template <int BLOCK, int T, int NCH, int TRIP>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(GMM_TILE_WPE, 8))) void em_tile_kernel(
    const float4 *__restrict__ pts,    // staged (x, y, z, tag), ntiles * T
    const float *__restrict__ cpar,    // K x 16 floats, then the bound C
    const float4 *__restrict__ shift,  // K
    double *__restrict__ part,         // grid rows of ncols
    float *__restrict__ lse_out,       // N or NULL
    TileArgs a) {
  using S = TileShape<BLOCK, T>;
  constexpr int G = S::G, TS = S::TS;
  constexpr int trip = TRIP;
  extern __shared__ __align__(16) unsigned char smem[];
  if (a.conv && (*a.conv & 1u)) return;   // converged fit: nothing to do
  const int K = a.K, KC = a.KC, P = a.P, mode = a.mode;
  float *E = reinterpret_cast<float *>(smem);
  float4 *Xs = reinterpret_cast<float4 *>(smem + tile_lds_bytes_e<BLOCK, T>(K, KC));
  float *reds = reinterpret_cast<float *>(Xs + TS);
  float *Mp = reds + G * T;
  double *wL = reinterpret_cast<double *>(Mp + T);

  const int tid = threadIdx.x;
  const int p = tid % T;
  // T is a multiple of the wave size, so g is wave-uniform; readfirstlane
  // makes that visible to the compiler: the component loops then run on
  // scalar registers with scalar loads of the parameter block.
  const int g = __builtin_amdgcn_readfirstlane(tid / T);
  const int b_lo = (g * K) / G;
  const int b_hi = ((g + 1) * K) / G;
  const bool mact = tid < KC * P;
  const int mb = mact ? tid % KC : 0;
  const int mq = mact ? tid / KC : 0;
  const double Cb = *reinterpret_cast<const double *>(cpar + (size_t)K * kParStride);

  float4 sh[NCH];
  double acc[NCH][kNStat];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int b = c * KC + mb;
    sh[c] = (b < K) ? shift[b] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int j = 0; j < kNStat; ++j) acc[c][j] = 0.0;
  }
  double Lacc = 0.0;
  // the zero pad columns of E and pad entries of Xs (read by the last subset)
  zero_pad<TS, T, BLOCK>(E, Xs, KC);

  // the next tile's point is loaded one tile ahead
  float4 xn = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
  if ((int)blockIdx.x < a.ntiles) xn = pts[(size_t)blockIdx.x * T + p];
  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const float4 x = xn;
    if (tile + (int)gridDim.x < a.ntiles)
      xn = pts[(size_t)(tile + gridDim.x) * T + p];
    const int tag = __float_as_int(x.w);
    const bool valid = tag >= 0;
    if (mode != kLabels) {
      float s = 0.0f;
      const float *q = cpar + (size_t)b_lo * kParStride;
      float *Ep = E + (size_t)b_lo * TS + p;
      int b = b_lo;
      if (NCH == 1) {
        for (; b + 4 <= b_hi; b += 4, q += 4 * kParStride, Ep += 4 * TS) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float e = __builtin_amdgcn_exp2f(
                comp_logterm(q + u * kParStride, x.x, x.y, x.z));
            Ep[u * TS] = e;
            s += e;
          }
        }
        for (; b < b_hi; ++b, q += kParStride, Ep += TS) {
          const float e = __builtin_amdgcn_exp2f(comp_logterm(q, x.x, x.y, x.z));
          *Ep = e;
          s += e;
        }
      } else {
        for (; b + 4 <= b_hi; b += 4, q += 4 * kParStride) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            s += __builtin_amdgcn_exp2f(
                comp_logterm(q + u * kParStride, x.x, x.y, x.z));
        }
        for (; b < b_hi; ++b, q += kParStride)
          s += __builtin_amdgcn_exp2f(comp_logterm(q, x.x, x.y, x.z));
      }
      reds[g * T + p] = s;
      __syncthreads();
      if (g == 0) {
        float st = reds[p];
#pragma unroll
        for (int j = 1; j < G; ++j) st += reds[j * T + p];
        float mref = 0.0f;
        if (valid && !(st >= 0x1p-100f)) {
          // far from every component: exact max-shifted sum for this point
          float m = -INFINITY;
          for (int bb = 0; bb < K; ++bb)
            m = fmaxf(m, comp_logterm(cpar + (size_t)bb * kParStride, x.x, x.y, x.z));
          st = 0.0f;
          for (int bb = 0; bb < K; ++bb) {
            const float e = __builtin_amdgcn_exp2f(
                comp_logterm(cpar + (size_t)bb * kParStride, x.x, x.y, x.z) - m);
            if (NCH == 1) E[bb * TS + p] = e;
            st += e;
          }
          mref = m;
        }
        Xs[p] = make_float4(x.x, x.y, x.z, valid ? __builtin_amdgcn_rcpf(st) : 0.0f);
        Mp[p] = mref;
        if (valid) {
          const double lse = (Cb + (double)mref + (double)__builtin_amdgcn_logf(st)) * kLn2;
          Lacc += lse;
          if (lse_out) lse_out[(size_t)tile * T + p] = (float)lse;
        }
      }
    } else if (NCH == 1) {
      for (int b = b_lo; b < b_hi; ++b) E[b * TS + p] = (b == tag) ? 1.0f : 0.0f;
      if (g == 0) Xs[p] = make_float4(x.x, x.y, x.z, valid ? 1.0f : 0.0f);
    } else if (g == 0) {
      Xs[p] = make_float4(x.x, x.y, x.z, valid ? 1.0f : 0.0f);
    }
    if (mode != kSoftLogLik) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int c0 = c * KC;
        if (NCH > 1) {
          __syncthreads();  // Xs / Mp ready; previous chunk consumed
          const int nc = min(KC, K - c0);
          const int lo = c0 + (g * nc) / G, hi = c0 + ((g + 1) * nc) / G;
          if (mode == kLabels) {
            for (int b = lo; b < hi; ++b)
              E[(b - c0) * TS + p] = (b == tag) ? 1.0f : 0.0f;
          } else {
            const float mref = Mp[p];
            for (int b = lo; b < hi; ++b)
              E[(b - c0) * TS + p] = __builtin_amdgcn_exp2f(
                  comp_logterm(cpar + (size_t)b * kParStride, x.x, x.y, x.z) - mref);
          }
        }
        __syncthreads();
        if (mact && c0 + mb < K)
          mstep_run<TRIP>(E + mb * TS + mq * trip, Xs + mq * trip, sh[c], acc[c]);
      }
    }
    __syncthreads();
  }

  // ---- this block's partial row
  double *row = part + (size_t)blockIdx.x * a.ncols;
  if (mode != kSoftLogLik) {
    // sum the P point subsets of each component, one statistic at a time
    double *D = reinterpret_cast<double *>(smem);  // P x KC
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
#pragma unroll
      for (int j = 0; j < kNStat; ++j) {
        __syncthreads();
        if (mact) D[mq * KC + mb] = acc[c][j];
        __syncthreads();
        for (int i = tid; i < KC; i += BLOCK) {
          const int b = c * KC + i;
          if (b < K) {
            double sum = 0.0;
            for (int qq = 0; qq < P; ++qq) sum += D[qq * KC + i];
            row[a.cmaj ? b * kNStat + j : j * K + b] = sum;
          }
        }
      }
    }
  }
  // block sum of the per-point log-normalisers (fixed order: DPP rows, then rows and waves in order)
  double v = Lacc;
  v = wave_sum_f64(v);
  if ((tid & 63) == 0) wL[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int j = 0; j < BLOCK / 64; ++j) sum += wL[j];
    row[kNStat * K] = sum;
  }

}

// ------------------------------------------------------ culled tile kernel
//
// Most tiles of a spatially ordered cloud lie far from most components:
// for those pairs 2^l'_pb underflows to exactly 0 in FP32 for every point,
// and the dense kernel spends its E- and M-work adding zeros.  The culled
// kernel skips such pairs with a conservative bound.  With the tile's
// bounding sphere (centre c, radius r) and P' = s P (|P'(x - mu)|^2 =
// log2(e)/2 (x - mu)^T Sigma^-1 (x - mu)),
//   |P'(x - mu)| >= |P'(c - mu)| - |P'|_F r   for every x in the sphere,
// so l'_pb <= c'_b - max(0, |P'(c - mu)| - |P'|_F r)^2.  When that is below
// kCullLog2 (2 units under the smallest FP32 subnormal exponent), e_pb
// rounds to 0 for every point of the tile and the pair is skipped: the
// result equals the dense kernel's up to the order of FP32 additions.
//
// A tile is T points (T / 64 point groups of one wave each).  Per tile:
//  cull      wave w tests components 64w .. 64w + 63 (parameters held in
//            registers for the whole launch) and stores the ballot; this is
//            done one tile ahead, at the end of the previous tile;
//  E-phase   the active components form an ordered list of slots; the
//            waves of a point group take every R-th slot and store e_pb in
//            LDS row `slot` (rows for SCAP slots; a tile with more active
//            components recomputes the later rows chunk by chunk);
//  normaliser  one thread per point: s_p, 1 / s_p, lse_p;
//  M-phase   lanes = (slot, point subset of TRIP points), the P subsets of
//            a slot in adjacent lanes: FP32 statistics, summed over the
//            subsets with DPP in a fixed order and added to FP64
//            per-component sums in LDS.
// A point with s_p below 2^-100 (far from every component) is left out of
// the M-phase and added afterwards, exactly as the dense kernel's fallback
// does it: its own maximum over all K components, one lane per component.
constexpr float kCullLog2 = -152.0f;

template <int BLOCK, int T, int TRIP, int SCAP>
struct CullShape {
  static constexpr int NW = BLOCK / 64;  // waves
  static constexpr int W = T / 64;       // point groups
  static constexpr int R = NW / W;       // waves per point group (E-phase)
  static constexpr int P = T / TRIP;     // point subsets per component
  static constexpr int XS = T + P;       // Xs entries (one pad per subset)
  static constexpr int RS = (T + P) | 1; // E row stride (odd)
  static_assert(T % 64 == 0 && NW % W == 0 && R >= 1, "tile and block");
  static_assert(P * TRIP == T && (P == 8 || P == 16), "subsets");
};

// LDS of the culled kernel for K components: E rows, Xs, shifts and cull
// parameters (unless CPR: then each lane holds its component's cull
// parameters in registers and the shifts are read from global memory),
// FP64 sums, masks, fallback (max, sum) per point, wL, partial normalisers,
// the active list and its length.
template <int BLOCK, int T, int TRIP, int SCAP, bool CPR = false>
__host__ __device__ constexpr size_t cull_lds_bytes(int K) {
  using S = CullShape<BLOCK, T, TRIP, SCAP>;
  return (((size_t)SCAP * S::RS * sizeof(float) + 15) & ~(size_t)15) +
         (size_t)S::XS * sizeof(float4) +
         (CPR ? (size_t)0 : (size_t)K * sizeof(float4)) +
         (CPR ? (size_t)0 : (size_t)((K + 63) / 64) * 64 * 3 * sizeof(float4)) +
         (size_t)K * kNStat * sizeof(double) + 32 * sizeof(uint64_t) +
         (size_t)S::W * sizeof(uint64_t) + (size_t)S::NW * sizeof(double) +
         (size_t)T * sizeof(float2) + (size_t)S::R * T * sizeof(float) +
         (size_t)2 * K * sizeof(uint16_t) + 16;
}

// Bounding sphere of every tile of tpts staged points: (centre, radius),
// radius < 0 for a tile of padding only.  One 256-thread block per tile.
__global__ __launch_bounds__(256) void tile_sphere_kernel(
    const float4 *__restrict__ pts, int tpts, float4 *__restrict__ sph) {
  __shared__ float sh[4][6];
  const int64_t t = blockIdx.x;
  float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY;
  float hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
  for (int i = threadIdx.x; i < tpts; i += 256) {
    const float4 x = pts[t * tpts + i];
    if (__float_as_int(x.w) >= 0) {
      lo0 = fminf(lo0, x.x); lo1 = fminf(lo1, x.y); lo2 = fminf(lo2, x.z);
      hi0 = fmaxf(hi0, x.x); hi1 = fmaxf(hi1, x.y); hi2 = fmaxf(hi2, x.z);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo0 = fminf(lo0, __shfl_xor(lo0, off, 64));
    lo1 = fminf(lo1, __shfl_xor(lo1, off, 64));
    lo2 = fminf(lo2, __shfl_xor(lo2, off, 64));
    hi0 = fmaxf(hi0, __shfl_xor(hi0, off, 64));
    hi1 = fmaxf(hi1, __shfl_xor(hi1, off, 64));
    hi2 = fmaxf(hi2, __shfl_xor(hi2, off, 64));
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[wv][0] = lo0; sh[wv][1] = lo1; sh[wv][2] = lo2;
    sh[wv][3] = hi0; sh[wv][4] = hi1; sh[wv][5] = hi2;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int v = 1; v < 4; ++v) {
    lo0 = fminf(lo0, sh[v][0]); lo1 = fminf(lo1, sh[v][1]); lo2 = fminf(lo2, sh[v][2]);
    hi0 = fmaxf(hi0, sh[v][3]); hi1 = fmaxf(hi1, sh[v][4]); hi2 = fmaxf(hi2, sh[v][5]);
  }
  if (!(lo0 <= hi0)) {
    sph[t] = make_float4(0.0f, 0.0f, 0.0f, -1.0f);
    return;
  }
  const float c0 = 0.5f * (lo0 + hi0), c1 = 0.5f * (lo1 + hi1),
              c2 = 0.5f * (lo2 + hi2);
  const float e0 = hi0 - lo0, e1 = hi1 - lo1, e2 = hi2 - lo2;
  // half diagonal, widened for the rounding of the centre and the norm
  const float scale = fmaxf(fmaxf(fabsf(c0), fabsf(c1)), fabsf(c2)) + 1.0f;
  const float r = 0.5f * sqrtf(e0 * e0 + e1 * e1 + e2 * e2) * (1.0f + 1e-5f) +
                  1e-5f * scale;
  sph[t] = make_float4(c0, c1, c2, r);
}

// v + the value of another lane (DPP, within rows of 16 lanes):
// xor 1, xor 2 (quad_perm), lane 7 - l of the half row, lane 15 - l of the
// row.  Applied in this order they sum 2, 4, 8 and 16 adjacent lanes.
__device__ __forceinline__ float dpp_add_xor1(float v) {
  return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_add_xor2(float v) {
  return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_add_half_mirror(float v) {
  return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_add_mirror(float v) {
  return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, true));
}

// Sum of the first NS statistics over the P adjacent lanes of a slot.
template <int P, int NS = kNStat>
__device__ __forceinline__ void subset_sum(float *a) {
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    a[j] = dpp_add_xor1(a[j]);
    a[j] = dpp_add_xor2(a[j]);
    a[j] = dpp_add_half_mirror(a[j]);
    if (P == 16) a[j] = dpp_add_mirror(a[j]);
  }
}

// Ten statistics summed over the 16 adjacent lanes of a slot as a
// reduce-scatter: each exchange keeps only the statistics that this lane's
// side of the pair will own, so lane q ends with the total of statistic
// scatter_stat(q) (-1: none). Exchanges: mirror (q, 15 - q) keeps 0-4 in
// the low half and 5-9 in the high half; half-mirror (q, 7 - q) keeps the
// first three / last two of those; then q ^ 2 and q ^ 1.
__device__ __forceinline__ int scatter_stat(int q) {
  const int r = q & 7, h = (q >> 3) * 5;
  return r < 3 ? h + r : (r == 4 || r == 5) ? h + r - 1 : -1;
}
__device__ __forceinline__ float dpp_from_mirror(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_from_half_mirror(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_from_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float scatter_sum16(const float *a, int q) {
  const bool hi = (q & 8) != 0, b4 = (q & 4) != 0, b2 = (q & 2) != 0, b1 = (q & 1) != 0;
  float k[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const float keep = hi ? a[j + 5] : a[j];
    const float send = hi ? a[j] : a[j + 5];
    k[j] = keep + dpp_from_mirror(send);
  }
  const float v0 = (b4 ? k[3] : k[0]) + dpp_from_half_mirror(b4 ? k[0] : k[3]);
  const float v1 = (b4 ? k[4] : k[1]) + dpp_from_half_mirror(b4 ? k[1] : k[4]);
  const float v2 = dpp_add_half_mirror(k[2]);
  const float w0 = dpp_add_xor2(v0), w1 = dpp_add_xor2(v1), w2 = dpp_add_xor2(v2);
  const float keep = b2 ? w2 : (b1 ? w1 : w0);
  const float send = b2 ? w2 : (b1 ? w0 : w1);
  return keep + dpp_from_xor1(send);
}

// Cull parameters of one component: (mu, c'), (P'0..3), (P'4, P'5, |P'|_F);
// c' = -inf for a lane past the last component.
struct CullPar {
  float4 u, v, z;
};

__device__ __forceinline__ CullPar cull_par(const float *__restrict__ cpar, int K, int c) {
  CullPar p;
  p.u = make_float4(0.f, 0.f, 0.f, -INFINITY);
  p.v = make_float4(0.f, 0.f, 0.f, 0.f);
  p.z = make_float4(0.f, 0.f, 0.f, 0.f);
  if (c < K) {
    const float *q = cpar + (size_t)c * kParStride;
    p.u = make_float4(q[0], q[1], q[2], q[3]);
    p.v = make_float4(q[4], q[5], q[6], q[7]);
    p.z = make_float4(q[8], q[9], q[10], 0.f);
  }
  return p;
}

// Cull test of one tile sphere (radius < 0: padding only) against one
// component.
__device__ __forceinline__ bool cull_test(float4 u, float4 v, float4 z, float4 sp) {
  const float d0 = sp.x - u.x, d1 = sp.y - u.y, d2 = sp.z - u.z;
  const float z0 = v.x * d0;
  const float z1 = fmaf(v.y, d0, v.z * d1);
  const float z2 = fmaf(v.w, d0, fmaf(z.x, d1, z.y * d2));
  const float dist = sqrtf(fmaf(z0, z0, fmaf(z1, z1, z2 * z2)));
  const float bnd = fmaxf(dist - z.z * sp.w, 0.0f);
  return fmaf(-bnd, bnd, u.w) >= kCullLog2;
}

// The wave's ballot of the cull test, this lane's component in registers
// or (3 float4) in LDS.
__device__ __forceinline__ uint64_t cull_ballot(const CullPar &cp, float4 sp) {
  return __ballot(sp.w >= 0.0f && cull_test(cp.u, cp.v, cp.z, sp));
}
__device__ __forceinline__ uint64_t cull_ballot(const float4 *cp, float4 sp) {
  bool act = false;
  if (sp.w >= 0.0f) act = cull_test(cp[0], cp[1], cp[2], sp);
  return __ballot(act);
}

#ifndef GMM_CULL_WPE
#define GMM_CULL_WPE 1
#endif
#ifndef GMM_CULL_EU
#define GMM_CULL_EU 8  // E-phase components per step
#endif

// LDS of the culled tile loop (carved from the dynamic shared memory).
struct CullLds {
  float *E;          // SCAP rows of RS
  float4 *Xs;        // XS
  float4 *ShL;       // K shifts (none if CPR)
  float4 *CP;        // cull parameters, 3 float4 per component, 64-padded
  double *acc;       // K x 10 FP64 sums
  uint64_t *masks;   // 2 x 16 (double-buffered: this tile's, the next)
  uint64_t *fbmask;  // W
  double *wL;        // NW
  float2 *fbv;       // T
  float *reds;       // R x T
  uint16_t *list;    // 2 x K component indices (K <= 1024)
  int *nact_s;       // 2
};

template <int BLOCK, int T, int TRIP, int SCAP, bool CPR>
__device__ __forceinline__ CullLds cull_carve(unsigned char *smem, int K) {
  using S = CullShape<BLOCK, T, TRIP, SCAP>;
  const int nchk = CPR ? 0 : (K + 63) >> 6;
  CullLds L;
  L.E = reinterpret_cast<float *>(smem);
  L.Xs = reinterpret_cast<float4 *>(
      smem + (((size_t)SCAP * S::RS * sizeof(float) + 15) & ~(size_t)15));
  L.ShL = L.Xs + S::XS;
  L.CP = L.ShL + (CPR ? 0 : K);
  L.acc = reinterpret_cast<double *>(L.CP + (size_t)nchk * 64 * 3);
  L.masks = reinterpret_cast<uint64_t *>(L.acc + (size_t)K * kNStat);
  L.fbmask = L.masks + 32;
  L.wL = reinterpret_cast<double *>(L.fbmask + S::W);
  L.fbv = reinterpret_cast<float2 *>(L.wL + S::NW);
  L.reds = reinterpret_cast<float *>(L.fbv + T);
  L.list = reinterpret_cast<uint16_t *>(L.reds + S::R * T);
  L.nact_s = reinterpret_cast<int *>(L.list + 2 * K);  // 2K uint16: 4-byte aligned
  return L;
}

// Per frame: shifts, cull parameters (unless CPR) and zero sums into LDS.
template <int BLOCK, bool CPR>
__device__ __forceinline__ void cull_begin(const CullLds &L, const float *__restrict__ cpar,
                                           const float4 *__restrict__ shift, int K) {
  const int tid = threadIdx.x;
  if (tid < 32) L.masks[tid] = 0;  // label passes OR into them
  for (int b = tid; b < K; b += BLOCK) {
    if (!CPR) L.ShL[b] = shift[b];
    for (int j = 0; j < kNStat; ++j) L.acc[(size_t)b * kNStat + j] = 0.0;
  }
  if (!CPR) {
    const int nchk = (K + 63) >> 6;
    for (int c = tid; c < nchk * 64; c += BLOCK) {
      const CullPar p = cull_par(cpar, K, c);
      L.CP[3 * c] = p.u;
      L.CP[3 * c + 1] = p.v;
      L.CP[3 * c + 2] = p.z;
    }
  }
  __syncthreads();
}

// The first tile's point of this lane and the first two tile spheres,
// loaded before the LDS staging so that both memory round trips overlap.
struct TilePre {
  float4 x, s0, s1;
};
template <int BLOCK, int T, int TRIP, int SCAP, bool LAB>
__device__ __forceinline__ TilePre tile_pre(const float4 *__restrict__ pts,
                                            const float4 *__restrict__ sph, int first, int end,
                                            int stride) {
  using S = CullShape<BLOCK, T, TRIP, SCAP>;
  const int w = threadIdx.x >> 6;
  const int t = (w % S::W) * 64 + (threadIdx.x & 63);
  TilePre p;
  p.x = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
  p.s0 = make_float4(0.f, 0.f, 0.f, -1.0f);
  p.s1 = p.s0;
  if (first < end) {
    p.x = pts[(size_t)first * T + t];
    if (!LAB) {
      p.s0 = sph[first];
      if (first + stride < end) p.s1 = sph[first + stride];
    }
  }
  return p;
}

// The tiles first, first + stride, ... < end of one frame: cull, E-phase,
// normaliser, M-phase into L.acc; lse sums into Lacc, active pairs into
// npairs (thread 0).
template <int BLOCK, int T, int TRIP, int SCAP, bool CPR, bool LAB, bool MEANS = false>
__device__ __forceinline__ void cull_tiles(
    const CullLds &L, const float4 *__restrict__ pts, const float4 *__restrict__ sph,
    const float *__restrict__ cpar, const float4 *__restrict__ shift, int K, int mode,
    int first, int end, int stride, float *__restrict__ lse_out, double &Lacc,
    unsigned long long &npairs, const TilePre &pre) {
  using S = CullShape<BLOCK, T, TRIP, SCAP>;
  constexpr int NW = S::NW, W = S::W, R = S::R, P = S::P, RS = S::RS;
  constexpr int SLOTS = BLOCK / P;  // slots per M round
  const int nchk = (K + 63) >> 6;
  float *E = L.E;
  float4 *Xs = L.Xs;
  const float4 *ShL = CPR ? shift : L.ShL;
  const float4 *CP = L.CP;
  double *acc = L.acc;
  uint64_t *masks = L.masks;
  uint64_t *fbmask = L.fbmask;
  float2 *fbv = L.fbv;
  float *reds = L.reds;
  uint16_t *list = L.list;
  int *nact_s = L.nact_s;

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int pg = w % W, rr = w / W;
  const int t = pg * 64 + lane;     // this lane's point in a tile
  const int tx = t + t / TRIP;      // its column in Xs and the E rows
  const double Cb = *reinterpret_cast<const double *>(cpar + (size_t)K * kParStride);
  // this lane's component in the cull (wave w < nchk tests chunk w)
  const int cc = (w << 6) + lane;
  CullPar creg;
  if constexpr (CPR) creg = cull_par(cpar, K, cc);
  auto cull_mask = [&](float4 sp) -> uint64_t {
    if constexpr (CPR) return cull_ballot(creg, sp);
    else return cull_ballot(CP + 3 * ((w << 6) + lane), sp);
  };
  // label passes: the components of a tile are the labels of its points
  // (masks zero beforehand; OR is order-free, so the list is deterministic).
  // One replica of the points; per wave one LDS OR per distinct label.
  auto mark_label = [&](float4 xq, uint64_t *mk) {
    if (rr != 0) return;
    const int tg = __float_as_int(xq.w);
    bool todo = tg >= 0;
    for (;;) {
      const uint64_t act = __ballot(todo);
      if (act == 0) break;
      const int first = __builtin_ctzll(act);
      const int t0 = __shfl(tg, first, 64);
      if (todo && tg == t0) todo = false;
      if (lane == first)
        atomicOr(reinterpret_cast<unsigned long long *>(mk + (t0 >> 6)), 1ull << (t0 & 63));
    }
  };

  // active list of a tile from masks buffer bf: chunk c is placed by wave
  // W + c when the block has that many waves (the waves of the first
  // replica are busy with the normaliser meanwhile), else by wave c
  const int wl = (NW >= W + nchk) ? w - W : w;
  auto build_list = [&](int bf) {
    const uint64_t *mk = masks + 16 * bf;
    if (wl >= 0 && wl < nchk) {
      int off = 0;
      for (int c = 0; c < wl; ++c) off += __popcll(mk[c]);
      const uint64_t m = mk[wl];
      const unsigned below = __builtin_amdgcn_mbcnt_hi(
          (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
      if ((m >> lane) & 1ull) list[K * bf + off + (int)below] = (uint16_t)((wl << 6) + lane);
      if (wl == nchk - 1 && lane == 0) nact_s[bf] = off + __popcll(m);
    }
  };

  // first tile: masks, list (buffer 0); the point and sphere of the next tile
  int tile = first;
  int cur = 0;
  float4 xn = pre.x;
  float4 spn = pre.s1;
  if (tile < end) {
    if constexpr (LAB) {
      mark_label(xn, masks);
    } else {
      if (w < nchk) {
        const uint64_t m = cull_mask(pre.s0);
        if (lane == 0) masks[w] = m;
      }
    }
  }
  __syncthreads();
  if (tile < end) build_list(0);
  __syncthreads();

  // Per tile three barriers: (E-phase + cull of the next tile) | A |
  // (normaliser + list of the next tile) | B | (M-phase [+ far points]) | C.
  // Masks and lists are double-buffered: `cur` is this tile's, `nxt` the
  // next tile's.
  for (; tile < end; tile += stride) {
    const float4 x = xn;
    const bool more = tile + stride < end;
    if (more) xn = pts[(size_t)(tile + stride) * T + t];
    const bool valid = __float_as_int(x.w) >= 0;
    const int nxt = cur ^ 1;
    const int nact = nact_s[cur];
    const uint16_t *lst = list + K * cur;

    if constexpr (LAB) {
      // ---- one-hot rows of the first SCAP slots; weight 1 per point
      const int tg = __float_as_int(x.w);
      for (int sl = rr; sl < min(nact, SCAP); sl += R)
        E[sl * RS + tx] = (__builtin_amdgcn_readfirstlane((int)lst[sl]) == tg) ? 1.0f : 0.0f;
      if (rr == 0) {
        Xs[tx] = make_float4(x.x, x.y, x.z, valid ? 1.0f : 0.0f);
        fbv[t] = make_float2(__int_as_float(tg), 0.0f);
        if (lane == 0) fbmask[pg] = 0;
      }
      // labels of the next tile (its mask buffer was cleared a tile ago)
      if (more) mark_label(xn, masks + 16 * nxt);
      __syncthreads();                                              // A
    } else {
      // ---- E-phase: slots rr, rr + R, ... of the active list, EU at a time
      float s = 0.0f;
      {
        constexpr int EU = GMM_CULL_EU;
        int sl = rr;
        for (; sl + (EU - 1) * R < nact; sl += EU * R) {
          float e[EU];
#pragma unroll
          for (int u = 0; u < EU; ++u) {
            const int b = __builtin_amdgcn_readfirstlane((int)lst[sl + u * R]);
            e[u] = __builtin_amdgcn_exp2f(
                comp_logterm(cpar + (size_t)b * kParStride, x.x, x.y, x.z));
          }
#pragma unroll
          for (int u = 0; u < EU; ++u) s += e[u];
          if (sl + (EU - 1) * R < SCAP) {
#pragma unroll
            for (int u = 0; u < EU; ++u) E[(sl + u * R) * RS + tx] = e[u];
          } else {
#pragma unroll
            for (int u = 0; u < EU - 1; ++u)
              if (sl + u * R < SCAP) E[(sl + u * R) * RS + tx] = e[u];
          }
        }
        for (; sl < nact; sl += R) {
          const int b0 = __builtin_amdgcn_readfirstlane((int)lst[sl]);
          const float e0 = __builtin_amdgcn_exp2f(
              comp_logterm(cpar + (size_t)b0 * kParStride, x.x, x.y, x.z));
          s += e0;
          if (sl < SCAP) E[sl * RS + tx] = e0;
        }
      }
      reds[rr * T + t] = s;
      // ---- cull of the next tile
      if (more && w < nchk) {
        const uint64_t m = cull_mask(spn);
        if (lane == 0) masks[16 * nxt + w] = m;
      }
      if (tile + 2 * stride < end) spn = sph[tile + 2 * stride];
      __syncthreads();                                              // A

      // ---- normaliser (waves of the first replica: one thread per point)
      if (rr == 0) {
        float st = reds[t];
#pragma unroll
        for (int j = 1; j < R; ++j) st += reds[j * T + t];
        const bool fb = valid && !(st >= 0x1p-100f);
        float mref = 0.0f;
        if (fb) {
          // far from every component: own maximum over all K (as the dense
          // kernel's fallback); the point joins the statistics afterwards
          float mx = -INFINITY;
          for (int bb = 0; bb < K; ++bb)
            mx = fmaxf(mx, comp_logterm(cpar + (size_t)bb * kParStride, x.x, x.y, x.z));
          st = 0.0f;
          for (int bb = 0; bb < K; ++bb)
            st += __builtin_amdgcn_exp2f(
                comp_logterm(cpar + (size_t)bb * kParStride, x.x, x.y, x.z) - mx);
          mref = mx;
          fbv[t] = make_float2(mx, st);
        }
        Xs[tx] = make_float4(x.x, x.y, x.z,
                             (valid && !fb) ? __builtin_amdgcn_rcpf(st) : 0.0f);
        const uint64_t fm = __ballot(fb);
        if (lane == 0) fbmask[pg] = fm;
        if (valid) {
          const double lse = (Cb + (double)mref + (double)__builtin_amdgcn_logf(st)) * kLn2;
          Lacc += lse;
          if (lse_out) lse_out[(size_t)tile * T + t] = (float)lse;
        }
      }
    }
    // ---- active list of the next tile
    if (more) build_list(nxt);
    __syncthreads();                                                // B

    // ---- M-phase over the active list, SCAP slots at a time
    if (tid == 0) npairs += (unsigned)nact;
    if (mode != kSoftLogLik) {
      const int q = tid % P;
      for (int c0 = 0; c0 < nact; c0 += SCAP) {
        const int nloc = min(SCAP, nact - c0);
        if (c0 > 0) {
          // rows of the slots [c0, c0 + nloc): recomputed, the normaliser is known
          __syncthreads();
          for (int u = w; u < nloc * W; u += NW) {
            const int sl = u / W, g2 = u % W;
            const int b = __builtin_amdgcn_readfirstlane((int)lst[c0 + sl]);
            const int t2 = g2 * 64 + lane, c2 = t2 + t2 / TRIP;
            if constexpr (LAB) {
              E[sl * RS + c2] = (__float_as_int(fbv[t2].x) == b) ? 1.0f : 0.0f;
            } else {
              const float4 xp = Xs[c2];
              E[sl * RS + c2] = __builtin_amdgcn_exp2f(
                  comp_logterm(cpar + (size_t)b * kParStride, xp.x, xp.y, xp.z));
            }
          }
          __syncthreads();
        }
        for (int s0 = 0; s0 < nloc; s0 += SLOTS) {
          const int sl = s0 + tid / P;
          if (sl < nloc) {
            const int b = lst[c0 + sl];
            const float4 sh = ShL[b];
            const float *Eb = E + sl * RS + q * (TRIP + 1);
            const float4 *Xb = Xs + q * (TRIP + 1);
            float av[kNStat];
#pragma unroll
            for (int j = 0; j < kNStat; ++j) av[j] = 0.0f;
#pragma unroll
            for (int j = 0; j < TRIP; ++j) {
              const float4 xr = Xb[j];
              const float gm = Eb[j] * xr.w;
              const float d0 = xr.x - sh.x, d1 = xr.y - sh.y, d2 = xr.z - sh.z;
              const float w0 = gm * d0, w1 = gm * d1, w2 = gm * d2;
              av[0] += gm;
              av[1] += w0; av[2] += w1; av[3] += w2;
              if constexpr (!MEANS) {
                av[4] = fmaf(w0, d0, av[4]);
                av[5] = fmaf(w1, d0, av[5]);
                av[6] = fmaf(w1, d1, av[6]);
                av[7] = fmaf(w2, d0, av[7]);
                av[8] = fmaf(w2, d1, av[8]);
                av[9] = fmaf(w2, d2, av[9]);
              }
            }
            // MEANS: the first pass of two-pass moments needs N and S1 only
            constexpr int NS = MEANS ? 4 : kNStat;
            double *ab = acc + (size_t)b * kNStat;
            if constexpr (P == 16 && NS == kNStat) {
              const float u0 = scatter_sum16(av, q);
              const int st = scatter_stat(q);
              if (st >= 0) ab[st] += (double)u0;
            } else {
              subset_sum<P, NS>(av);
              // lane q adds statistic q (and q + 8 when P = 8)
              float u0 = av[0];
#pragma unroll
              for (int j = 1; j < NS; ++j) u0 = (q == j) ? av[j] : u0;
              if (q < NS) ab[q] += (double)u0;
              if (!MEANS && P == 8 && q < 2) ab[q + 8] += (double)(q == 0 ? av[8] : av[9]);
            }
          }
        }
      }
    }

    // ---- far points of this tile (rare): wave 0, one lane per component,
    // after the M-phase's updates of the same sums
    bool anyfb = false;
#pragma unroll
    for (int g2 = 0; g2 < W; ++g2) anyfb = anyfb || fbmask[g2] != 0;
    if (mode != kSoftLogLik && anyfb) {
      __syncthreads();
      if (w == 0) {
        for (int g2 = 0; g2 < W; ++g2) {
          uint64_t fm = fbmask[g2];
          while (fm) {
            const int i = __builtin_ctzll(fm);
            fm &= fm - 1;
            const int t2 = g2 * 64 + i;
            const float4 xp = Xs[t2 + t2 / TRIP];
            const float2 v = fbv[t2];
            const float inv = __builtin_amdgcn_rcpf(v.y);
            for (int b = lane; b < K; b += 64) {
              const float gm = __builtin_amdgcn_exp2f(
                  comp_logterm(cpar + (size_t)b * kParStride, xp.x, xp.y, xp.z) - v.x) * inv;
              const float4 sh = ShL[b];
              const float d0 = xp.x - sh.x, d1 = xp.y - sh.y, d2 = xp.z - sh.z;
              double *ab = acc + (size_t)b * kNStat;
              ab[0] += (double)gm;
              ab[1] += (double)(gm * d0); ab[2] += (double)(gm * d1); ab[3] += (double)(gm * d2);
              ab[4] += (double)(gm * d0 * d0); ab[5] += (double)(gm * d1 * d0);
              ab[6] += (double)(gm * d1 * d1); ab[7] += (double)(gm * d2 * d0);
              ab[8] += (double)(gm * d2 * d1); ab[9] += (double)(gm * d2 * d2);
            }
          }
        }
      }
    }
    // label passes: this tile's mask buffer is marked again two tiles on
    if constexpr (LAB) {
      if (tid < 16) masks[16 * cur + tid] = 0;
    }
    __syncthreads();                                                // C
    cur = nxt;
  }
}

// The FP64 sums and the lse sum of one frame into its partial row.
// cmaj: the row in component-major order (the LDS order of the sums).
template <int BLOCK>
__device__ __forceinline__ void cull_end(const CullLds &L, double *__restrict__ row,
                                         int K, int mode, double Lacc, bool cmaj = false) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (mode != kSoftLogLik) {
    if (cmaj) {
      for (int i = tid; i < K * kNStat; i += BLOCK) row[i] = L.acc[i];
    } else {
      for (int i = tid; i < K * kNStat; i += BLOCK) {
        const int j = i / K, b = i - j * K;
        row[i] = L.acc[(size_t)b * kNStat + j];
      }
    }
  }
  double v = Lacc;
  v = wave_sum_f64(v);
  if (lane == 0) L.wL[w] = v;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int j = 0; j < BLOCK / 64; ++j) sum += L.wL[j];
    row[kNStat * K] = sum;
  }
  __syncthreads();  // LDS free for the next frame
}

// One tile pass of a single frame, grid-strided over the tiles.  LAB: the
// label pass (one-hot responsibilities from the staged labels; the active
// list of a tile is the set of its labels), a separate instantiation so
// that the soft passes carry none of its code.  MEANS: a soft pass that
// accumulates N and S1 only (the first pass of two-pass moments; the
// second-moment columns stay zero).
template <int BLOCK, int T, int TRIP, int SCAP, bool CPR, bool LAB, bool MEANS>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(GMM_CULL_WPE, 8))) void em_cull_kernel(
    const float4 *__restrict__ pts,    // staged (x, y, z, tag), ntiles * T
    const float4 *__restrict__ sph,    // ntiles bounding spheres
    const float *__restrict__ cpar,    // K x 16 floats, then the bound C
    const float4 *__restrict__ shift,  // K
    double *__restrict__ part,         // grid rows of ncols
    float *__restrict__ lse_out,       // N or NULL
    TileArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  // the flag, the first tile and the staged parameters are all requested
  // before the first wait; a converged fit returns before writing anything
  const bool done = a.conv && (*a.conv & 1u);
  const TilePre pre = tile_pre<BLOCK, T, TRIP, SCAP, LAB>(pts, sph, blockIdx.x, a.ntiles, gridDim.x);
  const CullLds L = cull_carve<BLOCK, T, TRIP, SCAP, CPR>(smem, a.K);
  cull_begin<BLOCK, CPR>(L, cpar, shift, a.K);
  if (done) return;   // uniform over the block, after cull_begin's barrier
  double Lacc = 0.0;
  unsigned long long npairs = 0;
  cull_tiles<BLOCK, T, TRIP, SCAP, CPR, LAB, MEANS>(L, pts, sph, cpar, shift, a.K, a.mode,
                                                   blockIdx.x, a.ntiles, gridDim.x, lse_out,
                                                   Lacc, npairs, pre);
  cull_end<BLOCK>(L, part + (size_t)blockIdx.x * a.ncols, a.K, a.mode, Lacc, a.cmaj != 0);
  if (threadIdx.x == 0 && a.pairs) atomicAdd(a.pairs, npairs);
}

// ------------------------------------------------------ reduction kernels
// Two fence-free launches after each tile pass:
//  reduce_rows_kernel  red2[y][c] = sum of part[r][c] over the y-th of
//                      gridDim.y chunks of rows; a block owns 64 columns x
//                      one chunk, its NT/64 waves take interleaved rows and
//                      are added in wave order (up to 16 loads in flight,
//                      adds in row order).
//  update_kernel       one block: tot[c] = sum_y red2[y][c] in y order, then
//                      the M-step (em_update_block) from LDS.
// Fits use kRedChunksFit chunks and 1024-thread reduce blocks: the single
// update block then has all of a thread's loads (4 columns x 4 rows) in
// flight at once.  Measured per 100-iteration fit at K = 100: 16 chunks
// 0.28 ms slower, 2 or 1 chunk 0.14 / 0.43 ms slower, 256-thread reduce
// blocks 0.07 ms slower.  The backward pass reduces into kRedChunks chunks.
constexpr int kRedChunks = 16;
constexpr int kRedChunksFit = 4;
constexpr int kUpdThreads = 1024;

template <int NT>
__global__ __launch_bounds__(NT) void reduce_rows_kernel(
    const double *__restrict__ part, int nrows, int ncols, int col0,
    double *__restrict__ red2, const unsigned *conv = nullptr) {
  if (conv && (*conv & 1u)) return;   // converged fit: nothing to do
  constexpr int NW = NT / 64;
  __shared__ double sh[NW][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = col0 + blockIdx.x * 64 + lane;
  const int cs = (nrows + (int)gridDim.y - 1) / (int)gridDim.y;
  const int r0 = blockIdx.y * cs, r1 = min(nrows, r0 + cs);
  double s = 0.0;
  if (c < ncols) {
    // the wave's rows r0 + wv + NW i: up to 16 loads in flight, added in order
    for (int base = r0 + wv; base < r1; base += 16 * NW) {
      double v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = base + NW * i;
        v[i] = r < r1 ? part[(size_t)r * ncols + c] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) s += v[i];
    }
  }
  sh[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && c < ncols) {
    double t = sh[0][lane];
#pragma unroll
    for (int j = 1; j < NW; ++j) t += sh[j][lane];
    red2[(size_t)blockIdx.y * ncols + c] = t;
  }
}

struct UpdArgs {
  int ncols, col0, K, mode, umode;
  double reg;
  double tol_abs;   // > 0: stop once |L(theta_t) - L(theta_t-1)| <= tol_abs
};
struct UpdPtrs {
  const double *red2;
  const float *cpar_in;
  const float4 *shift_in;
  float *cpar_out;
  float4 *shift_out;
  double *th64;
  double *loglik_slot;
  float *out_w, *out_mu, *out_cov;
  uint32_t *status;
  // fits with a tolerance: *conv is this pass's state (bit 0 converged,
  // bit 1 L_prev valid), read by every block; a full M-step writes the next
  // pass's state to *conv_next (a different word, so no block of the same
  // launch can see it) and L_prev to *Lprev.  NULL otherwise.
  unsigned *conv = nullptr;
  unsigned *conv_next = nullptr;
  double *Lprev = nullptr;
};

// tot = the column sums of red2 (LDS), the log-likelihood slot, then the
// M-step update; one block of kUpdThreads.
__device__ __forceinline__ void update_body(const UpdPtrs &q, const UpdArgs &a,
                                            unsigned char *smem) {
  const int tid = threadIdx.x;
  const int K = a.K;
  if (q.conv && (*q.conv & 1u)) {
    // converged: the iterations left are not run (their L is NaN); the
    // parameters carry over to the set the next pass reads
    if (tid == 0 && q.loglik_slot) q.loglik_slot[0] = (double)NAN;
    if (tid == 0 && q.conv_next) *q.conv_next = *q.conv;
    if (a.umode != kUpdNone) {
      for (int i = tid; i < (K + 1) * kParStride; i += kUpdThreads) q.cpar_out[i] = q.cpar_in[i];
      for (int b = tid; b < K; b += kUpdThreads) q.shift_out[b] = q.shift_in[b];
    }
    return;
  }
  double *tot = reinterpret_cast<double *>(smem);  // ncols
  double *scratch = tot + a.ncols;                 // 2 kUpdThreads / 64 + 2
  // four columns per thread at a time: all 16 loads in flight
  for (int c0 = a.col0 + tid; c0 < a.ncols; c0 += 4 * kUpdThreads) {
    double v[4][kRedChunksFit];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u * kUpdThreads;
#pragma unroll
      for (int y = 0; y < kRedChunksFit; ++y)
        v[u][y] = c < a.ncols ? q.red2[(size_t)y * a.ncols + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u * kUpdThreads;
      double t = 0.0;
#pragma unroll
      for (int y = 0; y < kRedChunksFit; ++y) t += v[u][y];
      if (c < a.ncols) tot[c] = t;
    }
  }
  __syncthreads();
  if (tid == 0 && q.loglik_slot && a.mode != kLabels) {
    const double L = tot[kNStat * K];
    q.loglik_slot[0] = L;
    if (!isfinite(L)) set_status(q.status, kStNonFinite);
  }
  if (a.umode != kUpdNone) {
    em_update_block<kUpdThreads>(tot, K, a.umode, a.reg, q.cpar_in, q.shift_in,
                                 q.cpar_out, q.shift_out, q.th64, scratch,
                                 q.status);
    // stopping rule, after a full M-step: theta_(t+1) is kept and the
    // following iterations are skipped once L changed by at most tol_abs
    if (tid == 0 && q.conv_next && a.umode == kUpdFull && a.mode == kSoftStats) {
      const double L = tot[kNStat * K];
      unsigned f = *q.conv;
      if ((f & 2u) && fabs(L - *q.Lprev) <= a.tol_abs) f |= 1u;
      *q.Lprev = L;
      *q.conv_next = f | 2u;
    }
  } else if (q.out_w) {
    for (int b = tid; b < K; b += kUpdThreads) {
      const double *t = q.th64 + (size_t)b * kTh64Stride;
      q.out_w[b] = (float)t[0];
      for (int j = 0; j < 3; ++j) q.out_mu[3 * b + j] = (float)t[1 + j];
      float *cv = q.out_cov + 9 * b;
      cv[0] = (float)t[4];
      cv[1] = cv[3] = (float)t[5];
      cv[4] = (float)t[6];
      cv[2] = cv[6] = (float)t[7];
      cv[5] = cv[7] = (float)t[8];
      cv[8] = (float)t[9];
    }
  }
}

// ------------------------------------------- fused reduction and M-step
// For lambda > 0 the M-step of a component needs no other component: the
// bound C is static (from lambda and K: c_b <= C + ln K), and sum_a N_a is
// n + K eps_N (each point's responsibilities sum to one).  The tile pass
// then writes its partial rows component-major (a component's ten sums
// adjacent), and one block per component sums its ten columns over the
// rows and updates it in FP64: thread (g, s) takes statistic s of the rows
// g, g + G, g + 2G, ...
// (G = kFuseGroups, added in row order), wave s adds the G group sums of
// statistic s (DPP row sums, then the four rows in order); block 0's last
// wave also sums the log-likelihood column (lane l the rows l, l + 64,
// ..., then the same wave sum).  One launch instead of reduce_rows_kernel
// + update_kernel, bitwise reproducible.
constexpr int kFuseGroups = 64;
static_assert(kFuseGroups == 64, "one group per lane of a statistic's wave");
constexpr int kFuseThreads = kNStat * kFuseGroups + 64;   // then one wave for L

struct FuseArgs {
  int K, ncols, nrows, mode, umode;
  double reg;
  double lnZ;      // ln(n + K eps_N) - 3/2 ln(lambda) - ln K: c_b - C = ln(N_b P00 P11 P22) - lnZ
  double Ntot;     // n + K eps_N
  double Chdr;     // C log2(e)
  double tol_abs;  // as UpdArgs
};

__global__ __launch_bounds__(kFuseThreads) void reduce_update_kernel(
    const double *__restrict__ part, UpdPtrs q, FuseArgs a) {
  __shared__ double sums[kFuseGroups * kNStat];
  __shared__ double tot[kNStat + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int K = a.K;
  const int b = blockIdx.x;
  if (q.conv && (*q.conv & 1u)) {
    // converged: nothing runs; the parameters carry over, L is NaN
    if (b == 0 && tid == 0 && q.loglik_slot) q.loglik_slot[0] = (double)NAN;
    if (b == 0 && tid == 0 && q.conv_next) *q.conv_next = *q.conv;
    if (a.umode != kUpdNone) {
      if (tid < kParStride)
        q.cpar_out[(size_t)b * kParStride + tid] = q.cpar_in[(size_t)b * kParStride + tid];
      if (tid == 0) q.shift_out[b] = q.shift_in[b];
      if (b == 0 && tid == 0)
        *reinterpret_cast<double *>(q.cpar_out + (size_t)K * kParStride) =
            *reinterpret_cast<const double *>(q.cpar_in + (size_t)K * kParStride);
    }
    return;
  }
  const bool lcol = b == 0 && a.mode != kLabels;
  const bool stats = a.mode != kSoftLogLik;
  constexpr int NS = kNStat * kFuseGroups;
  if (tid < NS) {
    if (stats) {
      const int g = tid / kNStat, st = tid - g * kNStat;
      const double *src = part + (size_t)b * kNStat + st;
      constexpr int G = kFuseGroups;
      // rounds of 16 rows, every load in flight (rows past the end add 0)
      double acc = 0.0;
      for (int r = g; r < a.nrows; r += 16 * G) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          v[u] = (r + u * G < a.nrows) ? src[(size_t)(r + u * G) * a.ncols] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += v[u];
      }
      sums[tid] = acc;
    }
  } else if (lcol) {
    const double *src = part + (size_t)kNStat * K;
    double acc = 0.0;
    for (int r = lane; r < a.nrows; r += 16 * 64) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        v[u] = (r + u * 64 < a.nrows) ? src[(size_t)(r + u * 64) * a.ncols] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += v[u];
    }
    acc = wave_sum_f64(acc);
    if (lane == 0) tot[kNStat] = acc;
  }
  // wave s adds the G = 64 group sums of statistic s (lane g: group g)
  __syncthreads();
  if (stats && (tid >> 6) < kNStat) {
    const double v = wave_sum_f64(sums[lane * kNStat + (tid >> 6)]);
    if (lane == 0) tot[tid >> 6] = v;
  }
  __syncthreads();
  if (lcol && tid == 0 && q.loglik_slot) {
    const double L = tot[kNStat];
    q.loglik_slot[0] = L;
    if (!isfinite(L)) set_status(q.status, kStNonFinite);
  }
  if (tid != 0) return;
  if (a.umode == kUpdNone) {
    if (q.out_w) {
      const double *t = q.th64 + (size_t)b * kTh64Stride;
      q.out_w[b] = (float)t[0];
      for (int j = 0; j < 3; ++j) q.out_mu[3 * b + j] = (float)t[1 + j];
      float *cv = q.out_cov + 9 * b;
      cv[0] = (float)t[4];
      cv[1] = cv[3] = (float)t[5];
      cv[4] = (float)t[6];
      cv[2] = cv[6] = (float)t[7];
      cv[5] = cv[7] = (float)t[8];
      cv[8] = (float)t[9];
    }
    return;
  }
  const double N0 = tot[0];
  const double S1[3] = {tot[1], tot[2], tot[3]};
  const float4 mf = q.shift_in[b];
  const double m[3] = {mf.x, mf.y, mf.z};
  const double Nb = N0 + kEpsN;
  const double rN = 1.0 / Nb;
  double mu[3], dl[3];
  for (int j = 0; j < 3; ++j) {
    mu[j] = (S1[j] + N0 * m[j]) * rN;
    dl[j] = mu[j] - m[j];
  }
  bool fin = isfinite(N0) && isfinite(S1[0]) && isfinite(S1[1]) && isfinite(S1[2]);
  if (a.umode == kUpdMeanOnly) {
    if (!fin) set_status(q.status, kStNonFinite);
    q.shift_out[b] = make_float4((float)mu[0], (float)mu[1], (float)mu[2], 0.0f);
    for (int j = 0; j < kParStride; ++j)
      q.cpar_out[(size_t)b * kParStride + j] = q.cpar_in[(size_t)b * kParStride + j];
    if (b == 0)
      *reinterpret_cast<double *>(q.cpar_out + (size_t)K * kParStride) =
          *reinterpret_cast<const double *>(q.cpar_in + (size_t)K * kParStride);
    return;
  }
  const int ij[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
  double C[6];
  for (int j = 0; j < 6; ++j) {
    const int r = ij[j][0], c = ij[j][1];
    const double s2 = tot[4 + j];
    const double v = s2 - S1[r] * dl[c] - dl[r] * S1[c] + N0 * dl[r] * dl[c];
    C[j] = v * rN + ((r == c) ? a.reg : 0.0);
    fin = fin && isfinite(s2);
  }
  if (!fin) set_status(q.status, kStNonFinite);
  double P[6];
  double cb = -INFINITY;
  if (chol_inv3(C, P)) cb = log(Nb * P[0] * P[2] * P[5]);
  if (!isfinite(cb)) set_status(q.status, kStNotSpd);
  double *t = q.th64 + (size_t)b * kTh64Stride;
  t[0] = Nb / a.Ntot;
  for (int j = 0; j < 3; ++j) t[1 + j] = mu[j];
  for (int j = 0; j < 6; ++j) t[4 + j] = C[j];
  t[10] = Nb;
  q.shift_out[b] = make_float4((float)mu[0], (float)mu[1], (float)mu[2], 0.0f);
  float *qq = q.cpar_out + (size_t)b * kParStride;
  if (isfinite(cb)) {
    store_eblock(qq, mu, P);
    qq[3] = (float)((cb - a.lnZ) * kLog2e);
  } else {
    qq[0] = (float)mu[0]; qq[1] = (float)mu[1]; qq[2] = (float)mu[2];
    for (int j = 0; j < 6; ++j) qq[4 + j] = 0.0f;
    qq[10] = 0.0f;
    qq[3] = -INFINITY;
  }
  if (b == 0) {
    *reinterpret_cast<double *>(q.cpar_out + (size_t)K * kParStride) = a.Chdr;
    // stopping rule (block 0 holds the log-likelihood column)
    if (q.conv_next && a.mode == kSoftStats) {
      const double L = tot[kNStat];
      unsigned f = *q.conv;
      if ((f & 2u) && fabs(L - *q.Lprev) <= a.tol_abs) f |= 1u;
      *q.Lprev = L;
      *q.conv_next = f | 2u;
    }
  }
}

__global__ __launch_bounds__(kUpdThreads) void update_kernel(UpdPtrs q, UpdArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  update_body(q, a, smem);
}

inline size_t update_lds_bytes(int K) {
  return ((size_t)kNStat * K + 1 + 2 * (kUpdThreads / 64) + 2) * sizeof(double);
}




// ---------------------------------------------------------- batched fits
// Many frames with their own N_f and K_f in one launch per M-phase class:
// the host cuts the concatenated tiles of the class's frames into one
// contiguous, cost-balanced range per block (cost = tiles x K_f), split into
// segments at frame boundaries; each segment writes one partial row of its
// frame.  A frame's rows are then added in row order by reduce_frames_kernel
// and update_frames_kernel runs one FP64 M-step per frame (one block each).
struct BFrame {
  long long poff;   // first double of the frame's partial rows
  long long toff;   // first staged tile
  int K;            // components
  int koff;         // first component (shift, FP64 state, outputs)
  int cpoff;        // first float of the frame's E-step block (K + 1 blocks)
  int P;            // M-phase point subsets
  int ncols;        // 10 K + 1
  int nrows;        // partial rows (segments)
  int roff;         // first column of the frame in the reduced array
  int n;            // points (the staged range is padded to 128)
};
struct BSeg {
  int frame, t0, t1, row;   // staged tiles [t0, t1) of one frame
};

// Batched fits: a block takes its segments (frame, tiles [t0, t1), row) in
// order, each with that frame's components (LDS sized for the largest K).
template <int BLOCK, int T, int TRIP, int SCAP>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(GMM_CULL_WPE, 8))) void em_cull_batch_kernel(
    const float4 *__restrict__ pts, const float4 *__restrict__ sph,
    const float *__restrict__ cpar_all, const float4 *__restrict__ shift_all,
    double *__restrict__ part, const BFrame *__restrict__ frames,
    const BSeg *__restrict__ segs, const int *__restrict__ blk_seg, int mode,
    int kmax) {
  extern __shared__ __align__(16) unsigned char smem[];
  const CullLds L = cull_carve<BLOCK, T, TRIP, SCAP, false>(smem, kmax);
  for (int si = blk_seg[blockIdx.x]; si < blk_seg[blockIdx.x + 1]; ++si) {
    const BSeg g = segs[si];
    const BFrame F = frames[g.frame];
    const float *cpar = cpar_all + F.cpoff;
    const TilePre pre = tile_pre<BLOCK, T, TRIP, SCAP, false>(pts, sph, g.t0, g.t1, 1);
    cull_begin<BLOCK, false>(L, cpar, shift_all + F.koff, F.K);
    double Lacc = 0.0;
    unsigned long long npairs = 0;
    cull_tiles<BLOCK, T, TRIP, SCAP, false, false>(L, pts, sph, cpar, shift_all + F.koff, F.K,
                                             mode, g.t0, g.t1, 1, nullptr, Lacc, npairs, pre);
    cull_end<BLOCK>(L, part + F.poff + (size_t)g.row * F.ncols, F.K, mode, Lacc);
  }
}


// Batched fits, dense: a block takes its segments (frame, tiles [t0, t1),
// row) in order, each with that frame's K and point-subset split P; every
// frame of one launch has the same TRIP = ceil(T / P) (LDS sized for the
// launch's largest K).
template <int BLOCK, int T, int TRIP>
__global__ __launch_bounds__(BLOCK) void em_batch_kernel(
    const float4 *__restrict__ pts, const float *__restrict__ cpar_all,
    const float4 *__restrict__ shift_all, double *__restrict__ part,
    const BFrame *__restrict__ frames, const BSeg *__restrict__ segs,
    const int *__restrict__ blk_seg, int mode, int kc_max) {
  using S = TileShape<BLOCK, T>;
  constexpr int G = S::G, TS = S::TS;
  extern __shared__ __align__(16) unsigned char smem[];
  float *E = reinterpret_cast<float *>(smem);
  float4 *Xs = reinterpret_cast<float4 *>(smem + tile_lds_bytes_e<BLOCK, T>(kc_max, kc_max));
  float *reds = reinterpret_cast<float *>(Xs + TS);
  double *wL = reinterpret_cast<double *>(reds + G * T + T);

  const int tid = threadIdx.x;
  const int p = tid % T;
  const int g = __builtin_amdgcn_readfirstlane(tid / T);
  zero_pad<TS, T, BLOCK>(E, Xs, kc_max);

  const int s0 = blk_seg[blockIdx.x], s1 = blk_seg[blockIdx.x + 1];
  for (int si = s0; si < s1; ++si) {
    const BSeg sg = segs[si];
    const BFrame F = frames[sg.frame];
    const int K = F.K, P = F.P;
    const float *cpar = cpar_all + F.cpoff;
    const double Cb = *reinterpret_cast<const double *>(cpar + (size_t)K * kParStride);
    const int b_lo = (g * K) / G;
    const int b_hi = ((g + 1) * K) / G;
    const bool mact = tid < K * P;
    const int mb = mact ? tid % K : 0;
    const int mq = mact ? tid / K : 0;
    const float4 sh = shift_all[F.koff + mb];
    double acc[kNStat];
#pragma unroll
    for (int j = 0; j < kNStat; ++j) acc[j] = 0.0;
    double Lacc = 0.0;
    for (int tile = sg.t0; tile < sg.t1; ++tile) {
      const float4 x = pts[(size_t)tile * T + p];
      const int tag = __float_as_int(x.w);
      const bool valid = tag >= 0;
      if (mode != kLabels) {
        float s = 0.0f;
        const float *q = cpar + (size_t)b_lo * kParStride;
        float *Ep = E + (size_t)b_lo * TS + p;
        int b = b_lo;
        for (; b + 4 <= b_hi; b += 4, q += 4 * kParStride, Ep += 4 * TS) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float e = __builtin_amdgcn_exp2f(
                comp_logterm(q + u * kParStride, x.x, x.y, x.z));
            Ep[u * TS] = e;
            s += e;
          }
        }
        for (; b < b_hi; ++b, q += kParStride, Ep += TS) {
          const float e = __builtin_amdgcn_exp2f(comp_logterm(q, x.x, x.y, x.z));
          *Ep = e;
          s += e;
        }
        reds[g * T + p] = s;
        __syncthreads();
        if (g == 0) {
          float st = reds[p];
#pragma unroll
          for (int j = 1; j < G; ++j) st += reds[j * T + p];
          float mref = 0.0f;
          if (valid && !(st >= 0x1p-100f)) {
            float m = -INFINITY;
            for (int bb = 0; bb < K; ++bb)
              m = fmaxf(m, comp_logterm(cpar + (size_t)bb * kParStride, x.x, x.y, x.z));
            st = 0.0f;
            for (int bb = 0; bb < K; ++bb) {
              const float e = __builtin_amdgcn_exp2f(
                  comp_logterm(cpar + (size_t)bb * kParStride, x.x, x.y, x.z) - m);
              E[bb * TS + p] = e;
              st += e;
            }
            mref = m;
          }
          Xs[p] = make_float4(x.x, x.y, x.z, valid ? __builtin_amdgcn_rcpf(st) : 0.0f);
          if (valid) Lacc += (Cb + (double)mref + (double)__builtin_amdgcn_logf(st)) * kLn2;
        }
      } else {
        for (int b = b_lo; b < b_hi; ++b) E[b * TS + p] = (b == tag) ? 1.0f : 0.0f;
        if (g == 0) Xs[p] = make_float4(x.x, x.y, x.z, valid ? 1.0f : 0.0f);
      }
      __syncthreads();
      if (mode != kSoftLogLik && mact)
        mstep_run<TRIP>(E + mb * TS + mq * TRIP, Xs + mq * TRIP, sh, acc);
      __syncthreads();
    }
    // this segment's row of its frame
    double *row = part + F.poff + (size_t)sg.row * F.ncols;
    if (mode != kSoftLogLik) {
      double *D = reinterpret_cast<double *>(smem);  // P x K
#pragma unroll
      for (int j = 0; j < kNStat; ++j) {
        __syncthreads();
        if (mact) D[mq * K + mb] = acc[j];
        __syncthreads();
        for (int i = tid; i < K; i += BLOCK) {
          double sum = 0.0;
          for (int qq = 0; qq < P; ++qq) sum += D[qq * K + i];
          row[j * K + i] = sum;
        }
      }
    }
    double v = Lacc;
    v = wave_sum_f64(v);
    if ((tid & 63) == 0) wL[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int j = 0; j < BLOCK / 64; ++j) sum += wL[j];
      row[kNStat * K] = sum;
    }
    __syncthreads();   // E, D and wL are reused by the next segment
    // D overwrote the start of E: restore the zero pad columns (the next
    // segment's first barrier orders these stores before any M-phase read)
    zero_pad<TS, T, BLOCK>(E, Xs, kc_max);
  }
}

template <int BLOCK, int T>
__host__ __device__ constexpr size_t batch_lds_bytes(int kc_max) {
  using S = TileShape<BLOCK, T>;
  return tile_lds_bytes_e<BLOCK, T>(kc_max, kc_max) + S::TS * sizeof(float4) +
         ((size_t)S::G * T + T) * sizeof(float) + (BLOCK / 64) * sizeof(double);
}

// red[frame roff + c] = sum over the frame's rows of part[row][c], rows
// added in order by 4 interleaved waves then in wave order.
__global__ __launch_bounds__(256) void reduce_frames_kernel(
    const double *__restrict__ part, const BFrame *__restrict__ frames,
    int only_L, double *__restrict__ red) {
  __shared__ double sh[4][64];
  const BFrame F = frames[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col0 = only_L ? kNStat * F.K : 0;
  const int c = col0 + blockIdx.y * 64 + lane;
  if (col0 + blockIdx.y * 64 >= F.ncols) return;   // uniform per block
  double s = 0.0;
  if (c < F.ncols) {
    const double *base = part + F.poff + c;
    int r = wv;
    for (; r + 12 < F.nrows; r += 16) {
      const double v0 = base[(size_t)r * F.ncols];
      const double v1 = base[(size_t)(r + 4) * F.ncols];
      const double v2 = base[(size_t)(r + 8) * F.ncols];
      const double v3 = base[(size_t)(r + 12) * F.ncols];
      s += v0; s += v1; s += v2; s += v3;
    }
    for (; r < F.nrows; r += 4) s += base[(size_t)r * F.ncols];
  }
  sh[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && c < F.ncols)
    red[F.roff + c] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

// One block per frame: the M-step of em_update_block on that frame's
// reduced columns (or, with kUpdNone, its log-likelihood and FP32 outputs).
__global__ __launch_bounds__(kUpdThreads) void update_frames_kernel(
    const double *__restrict__ red, const BFrame *__restrict__ frames,
    int mode, int umode, double reg, const float *cpar_in,
    const float4 *shift_in, float *cpar_out, float4 *shift_out, double *th64,
    double *loglik, int ll_stride, int ll_index, float *out_w, float *out_mu,
    float *out_cov, uint32_t *status) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BFrame F = frames[blockIdx.x];
  const int K = F.K, tid = threadIdx.x;
  double *tot = reinterpret_cast<double *>(smem);   // ncols
  double *scratch = tot + F.ncols;                  // kUpdThreads / 64 + 1
  const int col0 = (mode == kSoftLogLik) ? kNStat * K : 0;
  for (int c = col0 + tid; c < F.ncols; c += kUpdThreads) tot[c] = red[F.roff + c];
  __syncthreads();
  if (tid == 0 && loglik && mode != kLabels) {
    const double L = tot[kNStat * K];
    loglik[(size_t)blockIdx.x * ll_stride + ll_index] = L;
    if (!isfinite(L)) set_status(status, kStNonFinite);
  }
  double *t64 = th64 + (size_t)F.koff * kTh64Stride;
  if (umode != kUpdNone) {
    em_update_block<kUpdThreads>(tot, K, umode, reg, cpar_in + F.cpoff,
                                 shift_in + F.koff, cpar_out + F.cpoff,
                                 shift_out + F.koff, t64, scratch, status);
  } else if (out_w) {
    for (int b = tid; b < K; b += kUpdThreads) {
      const double *t = t64 + (size_t)b * kTh64Stride;
      const int gb = F.koff + b;
      out_w[gb] = (float)t[0];
      for (int j = 0; j < 3; ++j) out_mu[3 * gb + j] = (float)t[1 + j];
      float *cv = out_cov + 9 * gb;
      cv[0] = (float)t[4];
      cv[1] = cv[3] = (float)t[5];
      cv[4] = (float)t[6];
      cv[2] = cv[6] = (float)t[7];
      cv[5] = cv[7] = (float)t[8];
      cv[8] = (float)t[9];
    }
  }
}

// Caller-supplied theta_0 for every frame (one block per frame).
__global__ __launch_bounds__(kPreThreads) void precompute_frames_kernel(
    const float *__restrict__ w, const float *__restrict__ mu,
    const float *__restrict__ cov, const BFrame *__restrict__ frames,
    float *cpar_all, float4 *shift_all, double *th64, uint32_t *status) {
  __shared__ double scratch[kPreThreads];
  __shared__ double sC[GMM_MAX_K];
  const BFrame F = frames[blockIdx.x];
  float *cpar = cpar_all + F.cpoff;
  float4 *shift = shift_all + F.koff;
  double *t64 = th64 + (size_t)F.koff * kTh64Stride;
  for (int b = threadIdx.x; b < F.K; b += kPreThreads) {
    const int gb = F.koff + b;
    double pi = w[gb];
    double m[3] = {mu[3 * gb], mu[3 * gb + 1], mu[3 * gb + 2]};
    const float *c = cov + 9 * gb;
    double C[6] = {c[0], c[3], c[4], c[6], c[7], c[8]};
    if (!(pi > 0.0) || !isfinite(pi) || !isfinite(m[0]) || !isfinite(m[1]) ||
        !isfinite(m[2])) {
      set_status(status, kStBadArg);
      pi = 1.0;
    }
    const double cc = component_terms(b, pi, m, C, 0.0, cpar, shift, t64);
    if (!isfinite(cc)) set_status(status, kStNotSpd);
    sC[b] = cc;
  }
  apply_bound<kPreThreads>(F.K, sC, cpar, scratch);
}

// ------------------------------------------------------ registration backward
// Gradient of L = sum_n lse_n(y_n), y_n = R x_n + t (eq. 2-3 on the moved
// cloud), one launch over tiles like the forward:
//  E-phase per (point, component): as the forward, plus u = P'^T z'
//    (= s^2 Sigma_b^-1 d, s^2 = log2(e)/2) and G_p += e_pb u; after the
//    per-point normaliser s_p:  g_p = dL/dy_p = -G_p / (s^2 s_p).
//    dL/dx_p = R^T g_p is written per point; sum g_p and
//    sum (y_p - t) x g_p are accumulated per lane in FP64.
//  M-phase: the forward's statistics with the shift mu_b, i.e.
//    N_b, A_b = sum g d, B_b = sum g d d^T, d = y - mu_b.
// Row layout: the forward's 10 K + 1 columns, then sum g (3), sum (y-t) x g (3).
constexpr int kBwdExtra = 6;

template <int BLOCK, int T, int TRIP>
__global__ __launch_bounds__(BLOCK) void em_bwd_kernel(
    const float4 *__restrict__ pts, const float *__restrict__ cpar,
    const float4 *__restrict__ shift, const float *__restrict__ Rt,
    const double *__restrict__ grad_L, double *__restrict__ part,
    float *__restrict__ g_pts, TileArgs a, int64_t n_real) {
  using S = TileShape<BLOCK, T>;
  constexpr int G = S::G, TS = S::TS;
  constexpr int trip = TRIP;
  extern __shared__ __align__(16) unsigned char smem[];
  const int K = a.K, KC = a.KC, P = a.P;
  float *E = reinterpret_cast<float *>(smem);
  float4 *Xs = reinterpret_cast<float4 *>(smem + tile_lds_bytes_e<BLOCK, T>(K, KC));
  float *reds = reinterpret_cast<float *>(Xs + TS);   // G x T
  float *redg = reds + G * T;                           // 3 x G x T
  double *wL = reinterpret_cast<double *>(redg + 3 * G * T);  // 7 x BLOCK/64

  const int tid = threadIdx.x;
  const int p = tid % T;
  const int g = __builtin_amdgcn_readfirstlane(tid / T);
  const int b_lo = (g * K) / G;
  const int b_hi = ((g + 1) * K) / G;
  const bool mact = tid < KC * P;
  const int mb = mact ? tid % KC : 0;
  const int mq = mact ? tid / KC : 0;
  const double Cb = *reinterpret_cast<const double *>(cpar + (size_t)K * kParStride);
  const float inv_s2 = (float)(2.0 / kLog2e);
  const float gl = grad_L ? (float)grad_L[0] : 1.0f;
  float Rm[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
  float tv[3] = {0.f, 0.f, 0.f};
  if (Rt) {
    for (int i = 0; i < 9; ++i) Rm[i] = Rt[i];
    for (int i = 0; i < 3; ++i) tv[i] = Rt[9 + i];
  }

  const float4 sh = shift[mb];
  double acc[kNStat];
#pragma unroll
  for (int j = 0; j < kNStat; ++j) acc[j] = 0.0;
  double Lacc = 0.0, pg[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  zero_pad<TS, T, BLOCK>(E, Xs, KC);

  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const float4 x = pts[(size_t)tile * T + p];
    const bool valid = __float_as_int(x.w) >= 0;
    float s = 0.0f, G0 = 0.0f, G1 = 0.0f, G2 = 0.0f;
    for (int b = b_lo; b < b_hi; ++b) {
      const float *q = cpar + (size_t)b * kParStride;
      const float d0 = x.x - q[0], d1 = x.y - q[1], d2 = x.z - q[2];
      const float z0 = q[4] * d0;
      const float z1 = fmaf(q[5], d0, q[6] * d1);
      const float z2 = fmaf(q[7], d0, fmaf(q[8], d1, q[9] * d2));
      float l = fmaf(-z0, z0, q[3]);
      l = fmaf(-z1, z1, l);
      l = fmaf(-z2, z2, l);
      const float e = __builtin_amdgcn_exp2f(l);
      E[b * TS + p] = e;
      s += e;
      const float u0 = fmaf(q[4], z0, fmaf(q[5], z1, q[7] * z2));
      const float u1 = fmaf(q[6], z1, q[8] * z2);
      const float u2 = q[9] * z2;
      G0 = fmaf(e, u0, G0);
      G1 = fmaf(e, u1, G1);
      G2 = fmaf(e, u2, G2);
    }
    reds[g * T + p] = s;
    redg[(0 * G + g) * T + p] = G0;
    redg[(1 * G + g) * T + p] = G1;
    redg[(2 * G + g) * T + p] = G2;
    __syncthreads();
    if (g == 0) {
      float st = reds[p], H0 = redg[p], H1 = redg[G * T + p], H2 = redg[2 * G * T + p];
#pragma unroll
      for (int j = 1; j < G; ++j) {
        st += reds[j * T + p];
        H0 += redg[(0 * G + j) * T + p];
        H1 += redg[(1 * G + j) * T + p];
        H2 += redg[(2 * G + j) * T + p];
      }
      float mref = 0.0f;
      if (valid && !(st >= 0x1p-100f)) {
        // far from every component: redo the point with its own maximum
        float m = -INFINITY;
        for (int bb = 0; bb < K; ++bb)
          m = fmaxf(m, comp_logterm(cpar + (size_t)bb * kParStride, x.x, x.y, x.z));
        st = 0.0f; H0 = 0.0f; H1 = 0.0f; H2 = 0.0f;
        for (int bb = 0; bb < K; ++bb) {
          const float *q = cpar + (size_t)bb * kParStride;
          const float d0 = x.x - q[0], d1 = x.y - q[1], d2 = x.z - q[2];
          const float z0 = q[4] * d0;
          const float z1 = fmaf(q[5], d0, q[6] * d1);
          const float z2 = fmaf(q[7], d0, fmaf(q[8], d1, q[9] * d2));
          const float l = fmaf(-z2, z2, fmaf(-z1, z1, fmaf(-z0, z0, q[3])));
          const float e = __builtin_amdgcn_exp2f(l - m);
          E[bb * TS + p] = e;
          st += e;
          H0 = fmaf(e, fmaf(q[4], z0, fmaf(q[5], z1, q[7] * z2)), H0);
          H1 = fmaf(e, fmaf(q[6], z1, q[8] * z2), H1);
          H2 = fmaf(e, q[9] * z2, H2);
        }
        mref = m;
      }
      const float r = valid ? 1.0f / st : 0.0f;
      Xs[p] = make_float4(x.x, x.y, x.z, r);
      if (valid) {
        const double lse = (Cb + (double)mref + (double)log2f(st)) * kLn2;
        Lacc += lse;
        // g = dL/dy = -Sigma^-1 d weighted = -(H / s_p) / s^2
        const float c = -r * inv_s2;
        const float g0 = c * H0, g1 = c * H1, g2 = c * H2;
        const size_t idx = (size_t)tile * T + p;
        if (g_pts && idx < (size_t)n_real) {
          g_pts[3 * idx + 0] = gl * (Rm[0] * g0 + Rm[3] * g1 + Rm[6] * g2);
          g_pts[3 * idx + 1] = gl * (Rm[1] * g0 + Rm[4] * g1 + Rm[7] * g2);
          g_pts[3 * idx + 2] = gl * (Rm[2] * g0 + Rm[5] * g1 + Rm[8] * g2);
        }
        const float rx = x.x - tv[0], ry = x.y - tv[1], rz = x.z - tv[2];
        pg[0] += g0; pg[1] += g1; pg[2] += g2;
        pg[3] += (double)(ry * g2 - rz * g1);
        pg[4] += (double)(rz * g0 - rx * g2);
        pg[5] += (double)(rx * g1 - ry * g0);
      }
    }
    __syncthreads();
    if (mact && mb < K)
      mstep_run<TRIP>(E + mb * TS + mq * trip, Xs + mq * trip, sh, acc);
    __syncthreads();
  }

  double *row = part + (size_t)blockIdx.x * a.ncols;
  double *D = reinterpret_cast<double *>(smem);  // P x KC
#pragma unroll
  for (int j = 0; j < kNStat; ++j) {
    __syncthreads();
    if (mact) D[mq * KC + mb] = acc[j];
    __syncthreads();
    for (int i = tid; i < K; i += BLOCK) {
      double sum = 0.0;
      for (int qq = 0; qq < P; ++qq) sum += D[qq * KC + i];
      row[j * K + i] = sum;
    }
  }
  // block sums of lse and the six pose terms (fixed order: DPP rows, then rows and waves in order)
  double vals[7] = {Lacc, pg[0], pg[1], pg[2], pg[3], pg[4], pg[5]};
  for (int k = 0; k < 7; ++k) {
    double v = vals[k];
    v = wave_sum_f64(v);
    if ((tid & 63) == 0) wL[k * (BLOCK / 64) + (tid >> 6)] = v;
  }
  __syncthreads();
  if (tid < 7) {
    double sum = 0.0;
    for (int j = 0; j < BLOCK / 64; ++j) sum += wL[tid * (BLOCK / 64) + j];
    row[kNStat * K + tid] = sum;
  }
}

template <int BLOCK, int T>
__host__ __device__ constexpr size_t bwd_lds_bytes(int K) {
  using S = TileShape<BLOCK, T>;
  return tile_lds_bytes_e<BLOCK, T>(K, K) + S::TS * sizeof(float4) +
         4 * (size_t)S::G * T * sizeof(float) + 7 * (BLOCK / 64) * sizeof(double);
}

// Final step of the backward (one block): from the reduced columns and the
// FP32 mixture (Sigma^-1 = P^T P from an FP64 Cholesky),
//   dL/dpi_b = N_b / pi_b,  dL/dmu_b = Sigma^-1 A_b,
//   dL/dSigma_b = 1/2 Sigma^-1 B_b Sigma^-1 - 1/2 N_b Sigma^-1,
//   dL/dt = sum g,  dL/domega = J_l^T sum (y - t) x g,
// all times grad_L.
__global__ __launch_bounds__(256) void bwd_finish_kernel(
    const double *__restrict__ red2, int ncols, int K,
    const float *__restrict__ w, const float *__restrict__ cov,
    const double *__restrict__ pose64, const double *__restrict__ grad_L,
    float *g_pose6, float *g_w, float *g_mu, float *g_cov, uint32_t *status) {
  const double gl = grad_L ? grad_L[0] : 1.0;
  auto col = [&](int c) {
    double t = 0.0;
#pragma unroll
    for (int y = 0; y < kRedChunks; ++y) t += red2[(size_t)y * ncols + c];
    return t;
  };
  for (int b = threadIdx.x; b < K; b += blockDim.x) {
    const double N = col(b);
    const double A[3] = {col(K + b), col(2 * K + b), col(3 * K + b)};
    double Bl[6];
    for (int j = 0; j < 6; ++j) Bl[j] = col((4 + j) * K + b);
    const float *c = cov + 9 * b;
    const double C[6] = {c[0], c[3], c[4], c[6], c[7], c[8]};
    double L[6], P[6];
    if (!chol3(C, L)) {
      // no gradient exists: the component's outputs are NaN, not stale memory
      set_status(status, kStNotSpd);
      const float nan = __builtin_nanf("");
      if (g_w) g_w[b] = nan;
      if (g_mu)
        for (int i = 0; i < 3; ++i) g_mu[3 * b + i] = nan;
      if (g_cov)
        for (int i = 0; i < 9; ++i) g_cov[9 * b + i] = nan;
      continue;
    }
    tri_inv3(L, P);
    // Sigma^-1 = P^T P (full symmetric)
    const double Pm[9] = {P[0], 0.0, 0.0, P[1], P[2], 0.0, P[3], P[4], P[5]};
    double Si[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double v = 0.0;
        for (int k = 0; k < 3; ++k) v += Pm[k * 3 + i] * Pm[k * 3 + j];
        Si[i * 3 + j] = v;
      }
    const double B[9] = {Bl[0], Bl[1], Bl[3], Bl[1], Bl[2], Bl[4], Bl[3], Bl[4], Bl[5]};
    if (g_w) g_w[b] = (float)(gl * N / (double)w[b]);
    if (g_mu)
      for (int i = 0; i < 3; ++i)
        g_mu[3 * b + i] = (float)(gl * (Si[i * 3] * A[0] + Si[i * 3 + 1] * A[1] + Si[i * 3 + 2] * A[2]));
    if (g_cov) {
      double T1[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double v = 0.0;
          for (int k = 0; k < 3; ++k) v += Si[i * 3 + k] * B[k * 3 + j];
          T1[i * 3 + j] = v;
        }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double v = 0.0;
          for (int k = 0; k < 3; ++k) v += T1[i * 3 + k] * Si[k * 3 + j];
          g_cov[9 * b + i * 3 + j] = (float)(gl * (0.5 * v - 0.5 * N * Si[i * 3 + j]));
        }
    }
  }
  if (threadIdx.x == 0 && g_pose6) {
    const int c0 = kNStat * K + 1;
    const double gs[3] = {col(c0), col(c0 + 1), col(c0 + 2)};
    const double h[3] = {col(c0 + 3), col(c0 + 4), col(c0 + 5)};
    double J[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (pose64)
      for (int i = 0; i < 9; ++i) J[i] = pose64[12 + i];
    for (int i = 0; i < 3; ++i) {
      g_pose6[i] = (float)(gl * (J[i] * h[0] + J[3 + i] * h[1] + J[6 + i] * h[2]));
      g_pose6[3 + i] = (float)(gl * gs[i]);
    }
    if (!isfinite(gs[0] + gs[1] + gs[2] + h[0] + h[1] + h[2]))
      set_status(status, kStNonFinite);
  }
}

}  // namespace gmm_dev
