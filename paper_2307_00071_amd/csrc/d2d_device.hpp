// Distribution-to-distribution registration of two Gaussian mixtures
// (device code, included by d2d.hip): the paper's GIRA Registration (Sec.
// IV), anisotropic and isoplanar variants and the isoplanar-then-
// anisotropic hybrid, which the paper names without formulas.  The reading
// implemented:
//   f(T) = ln sum_ij pi_i tau_j N(R mu_i + t; nu_j, R Sigma_i R^T + Lambda_j)
// (the log of the integral of the product of the transformed source density
// and the target density), maximised over T = (R, t) by Newton-type steps
// in left-perturbation coordinates (delta, dt): curvature = the Gauss-Newton
// matrix H = sum_ij gamma_ij J^T S_ij^-1 J (J = [-[R mu_i]_x, I], S held at
// T), right-hand side = the exact gradient, x = H^-1 grad f, and the first
// of the trial poses R' = exp([s x_w]_x) R, t' = t + s x_t, s = 1, 1/2, ...,
// 2^-7, that increases f.  Isoplanar covariances are I - (1 - 1e-3) v v^T,
// v the eigenvector of the smallest eigenvalue.
//
// Everything is FP64: the pair terms are few (M N, up to a few 1e6) and the
// step compares f between poses.  Pairs are processed by one block per
// (source component, pose), threads over the target components; every sum
// is a fixed-order reduction (per thread in j order, a butterfly per wave,
// waves in order, blocks in order), so results are bitwise reproducible.
// The optimisation never synchronises with the host: each iteration's
// kernels read a device "stopped" flag and return at once when the stage has
// ended.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gmm.h"

namespace d2d_dev {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kTrials = 8;          // step sizes 1, 1/2, ..., 2^-7
constexpr int kPose = 12;           // R row-major (9), t (3)
constexpr int kNStat = 27;          // H: delta-delta 6, delta-t 9, t-t 6; grad 6
constexpr double kIsoEps = 1e-3;
constexpr double kStepTol = 1e-8;
constexpr double kLn2Pi = 1.83787706640934548356;

constexpr uint32_t kStBadArg = 1u << GMM_ERR_INVALID_ARG;
constexpr uint32_t kStNotSpd = 1u << GMM_ERR_NOT_SPD;
constexpr uint32_t kStNonFinite = 1u << GMM_ERR_NONFINITE;

// Device state; the status word first (gmm_workspace_status reads it).
struct State {
  uint32_t status;
  int stopped;        // the current stage has ended
  int stage;          // 0 isoplanar, 1 anisotropic
  int hist_n;         // history entries written
  int count[2];       // accepted iterations per stage
  int pad[2];
  double pose[1 + kTrials][kPose];   // [0] current, [1 ..] trials
  double fval[1 + kTrials];          // f at those poses
  double f;                          // f at the current pose
  double grad[6];                    // df/d(delta, dt) at the current pose
};

// A mixture in FP64: ln w, mean, covariance lower triangle (00 10 11 20 21 22).
struct Mix {
  const double *lw;
  const double *mu;
  const double *cov;
  int n;
};

__device__ inline void set_status(uint32_t *st, uint32_t bits) { atomicOr(st, bits); }

// Rodrigues' formula (series below |w| = 1e-4), row-major R.
__device__ inline void expso3(const double *w, double *R) {
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = sqrt(th2);
  double a, b;
  if (th < 1e-4) {
    a = 1.0 - th2 / 6.0;
    b = 0.5 - th2 / 24.0;
  } else {
    a = sin(th) / th;
    b = (1.0 - cos(th)) / th2;
  }
  const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double kk = 0.0;
      for (int m = 0; m < 3; ++m) kk += K[3 * r + m] * K[3 * m + c];
      R[3 * r + c] = (r == c ? 1.0 : 0.0) + a * K[3 * r + c] + b * kk;
    }
}

// Left Jacobian of SO(3), row-major.
__device__ inline void left_jacobian(const double *w, double *J) {
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = sqrt(th2);
  double a, b;
  if (th < 1e-4) {
    a = 0.5 - th2 / 24.0;
    b = 1.0 / 6.0 - th2 / 120.0;
  } else {
    a = (1.0 - cos(th)) / th2;
    b = (th - sin(th)) / (th2 * th);
  }
  const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double kk = 0.0;
      for (int m = 0; m < 3; ++m) kk += K[3 * r + m] * K[3 * m + c];
      J[3 * r + c] = (r == c ? 1.0 : 0.0) + a * K[3 * r + c] + b * kk;
    }
}

// Eigenvector of the smallest eigenvalue of a symmetric 3 x 3 matrix
// (lower triangle), cyclic Jacobi rotations.
__device__ inline void smallest_eigvec(const double *c6, double *v) {
  double A[3][3] = {{c6[0], c6[1], c6[3]}, {c6[1], c6[2], c6[4]}, {c6[3], c6[4], c6[5]}};
  double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
    const double scale = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
    if (!(off > 1e-18 * scale)) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {   // A <- A G
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {   // A <- G^T A
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {   // V <- V G
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  int m = 0;
  if (A[1][1] < A[m][m]) m = 1;
  if (A[2][2] < A[m][m]) m = 2;
  const double n = sqrt(V[0][m] * V[0][m] + V[1][m] * V[1][m] + V[2][m] * V[2][m]);
  for (int k = 0; k < 3; ++k) v[k] = V[k][m] / n;
}

// FP64 copies of one mixture: ln w, mean, covariance (isoplanar when iso).
__global__ __launch_bounds__(kThreads) void d2d_prep_kernel(
    const float *__restrict__ w, const float *__restrict__ mu,
    const float *__restrict__ cov, int n, int iso, double *__restrict__ lw,
    double *__restrict__ mu64, double *__restrict__ cov64, uint32_t *status) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= n) return;
  const double wk = w[k];
  if (!(wk > 0.0) || !isfinite(wk)) set_status(status, kStBadArg);
  lw[k] = log(wk);
  for (int j = 0; j < 3; ++j) {
    mu64[3 * k + j] = mu[3 * k + j];
    if (!isfinite(mu64[3 * k + j])) set_status(status, kStNonFinite);
  }
  const float *c = cov + 9 * k;
  double c6[6] = {c[0], c[3], c[4], c[6], c[7], c[8]};
  if (iso) {
    double v[3];
    smallest_eigvec(c6, v);
    const double a = 1.0 - kIsoEps;
    c6[0] = 1.0 - a * v[0] * v[0];
    c6[1] = -a * v[1] * v[0];
    c6[2] = 1.0 - a * v[1] * v[1];
    c6[3] = -a * v[2] * v[0];
    c6[4] = -a * v[2] * v[1];
    c6[5] = 1.0 - a * v[2] * v[2];
  }
  for (int j = 0; j < 6; ++j) cov64[6 * k + j] = c6[j];
}

// The state at the start of a call: pose from the 4 x 4 transform or from
// (omega, t); history cleared to NaN.
__global__ void d2d_init_kernel(State *st, const double *T0, const double *pose6,
                                double *hist, int hist_len, int *counts) {
  const int tid = threadIdx.x;
  for (int i = tid; i < hist_len; i += blockDim.x) hist[i] = (double)NAN;
  if (tid != 0) return;
  st->status = 0u;
  st->stopped = 0;
  st->stage = 0;
  st->hist_n = 0;
  st->count[0] = st->count[1] = 0;
  double *p = st->pose[0];
  if (T0) {
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) p[3 * r + c] = T0[4 * r + c];
      p[9 + r] = T0[4 * r + 3];
    }
  } else {
    expso3(pose6, p);
    for (int r = 0; r < 3; ++r) p[9 + r] = pose6[3 + r];
  }
  bool fin = true;
  for (int i = 0; i < kPose; ++i) fin = fin && isfinite(p[i]);
  if (!fin) set_status(&st->status, kStNonFinite);
  if (counts) counts[0] = counts[1] = 0;
}

// A new stage: the flag cleared.
__global__ void d2d_stage_kernel(State *st, int stage) {
  if (threadIdx.x == 0) {
    st->stopped = 0;
    st->stage = stage;
  }
}

// The source component's transformed mean a = R mu_i, a + t and
// Sigma' = R Sigma_i R^T (lower triangle).
struct SrcTerms {
  double a[3], at[3], Sp[6];
};

__device__ inline void src_terms(const double *P, const double *mu, const double *c6,
                                 SrcTerms *o) {
  const double C[9] = {c6[0], c6[1], c6[3], c6[1], c6[2], c6[4], c6[3], c6[4], c6[5]};
  double RC[9];
  for (int r = 0; r < 3; ++r) {
    o->a[r] = P[3 * r] * mu[0] + P[3 * r + 1] * mu[1] + P[3 * r + 2] * mu[2];
    o->at[r] = o->a[r] + P[9 + r];
    for (int c = 0; c < 3; ++c)
      RC[3 * r + c] = P[3 * r] * C[c] + P[3 * r + 1] * C[3 + c] + P[3 * r + 2] * C[6 + c];
  }
  const int ij[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
  for (int e = 0; e < 6; ++e) {
    const int r = ij[e][0], c = ij[e][1];
    o->Sp[e] = RC[3 * r] * P[3 * c] + RC[3 * r + 1] * P[3 * c + 1] + RC[3 * r + 2] * P[3 * c + 2];
  }
}

// One pair: S = Sigma' + Lambda_j, its Cholesky factor L, z = L^-1 d and
// ell; false when S is not positive definite.
struct PairTerms {
  double L[6];   // 00 10 11 20 21 22
  double d[3], z[3];
  double ell;
};

__device__ inline bool pair_terms(const SrcTerms &s, double lwi, const double *nu,
                                  const double *lam, double lwj, PairTerms *p) {
  const double S0 = s.Sp[0] + lam[0], S1 = s.Sp[1] + lam[1], S2 = s.Sp[2] + lam[2];
  const double S3 = s.Sp[3] + lam[3], S4 = s.Sp[4] + lam[4], S5 = s.Sp[5] + lam[5];
  if (!(S0 > 0.0)) return false;
  const double l00 = sqrt(S0);
  const double l10 = S1 / l00, l20 = S3 / l00;
  const double q11 = S2 - l10 * l10;
  if (!(q11 > 0.0)) return false;
  const double l11 = sqrt(q11);
  const double l21 = (S4 - l20 * l10) / l11;
  const double q22 = S5 - l20 * l20 - l21 * l21;
  if (!(q22 > 0.0)) return false;
  const double l22 = sqrt(q22);
  p->L[0] = l00; p->L[1] = l10; p->L[2] = l11; p->L[3] = l20; p->L[4] = l21; p->L[5] = l22;
  for (int k = 0; k < 3; ++k) p->d[k] = s.at[k] - nu[k];
  p->z[0] = p->d[0] / l00;
  p->z[1] = (p->d[1] - l10 * p->z[0]) / l11;
  p->z[2] = (p->d[2] - l20 * p->z[0] - l21 * p->z[1]) / l22;
  const double quad = p->z[0] * p->z[0] + p->z[1] * p->z[1] + p->z[2] * p->z[2];
  p->ell = lwi + lwj - 1.5 * kLn2Pi - log(l00 * l11 * l22) - 0.5 * quad;
  return true;
}

// (m, s) pairs: the log-sum-exp m + ln s, merged exactly as written.
__device__ inline void lse_merge(double &m, double &s, double m2, double s2) {
  if (s2 == 0.0) return;
  if (s == 0.0) {
    m = m2;
    s = s2;
    return;
  }
  if (m2 > m) {
    s = s * exp(m - m2) + s2;
    m = m2;
  } else {
    s = s + s2 * exp(m2 - m);
  }
}

// Value pass: f at pose p0 + blockIdx.y; rows[(p, i)] = (m, s) of source
// component i = blockIdx.x against every target component.
__global__ __launch_bounds__(kThreads) void d2d_value_kernel(
    Mix src, Mix tgt, State *st, int p0, double *__restrict__ rows) {
  if (st->stopped) return;
  __shared__ double wm[kWaves], ws[kWaves];
  const int i = blockIdx.x, p = p0 + blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  SrcTerms s;
  src_terms(st->pose[p], src.mu + 3 * i, src.cov + 6 * i, &s);
  const double lwi = src.lw[i];
  double m = 0.0, sm = 0.0;
  bool bad = false;
  for (int j = tid; j < tgt.n; j += kThreads) {
    PairTerms q;
    if (!pair_terms(s, lwi, tgt.mu + 3 * j, tgt.cov + 6 * j, tgt.lw[j], &q)) {
      bad = true;
      continue;
    }
    lse_merge(m, sm, q.ell, 1.0);
  }
  if (bad) set_status(&st->status, kStNotSpd);
  for (int off = 32; off > 0; off >>= 1) {
    const double m2 = __shfl_xor(m, off, 64), s2 = __shfl_xor(sm, off, 64);
    lse_merge(m, sm, m2, s2);
  }
  if (lane == 0) {
    wm[wv] = m;
    ws[wv] = sm;
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < kWaves; ++k) lse_merge(m, sm, wm[k], ws[k]);
    double *r = rows + 2 * ((size_t)blockIdx.y * src.n + i);
    r[0] = m;
    r[1] = sm;
  }
}

// fval[p0 + blockIdx.x] = the log-sum-exp of the pose's M rows: thread t
// merges rows t, t + 256, ... in order, then waves and the block in order.
__global__ __launch_bounds__(kThreads) void d2d_value_reduce_kernel(
    State *st, int p0, const double *__restrict__ rows, int M) {
  if (st->stopped) return;
  __shared__ double wm[kWaves], ws[kWaves];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double *r = rows + 2 * (size_t)blockIdx.x * M;
  double m = 0.0, s = 0.0;
  for (int i = tid; i < M; i += kThreads) lse_merge(m, s, r[2 * i], r[2 * i + 1]);
  for (int off = 32; off > 0; off >>= 1) {
    const double m2 = __shfl_xor(m, off, 64), s2 = __shfl_xor(s, off, 64);
    lse_merge(m, s, m2, s2);
  }
  if (lane == 0) {
    wm[wv] = m;
    ws[wv] = s;
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < kWaves; ++k) lse_merge(m, s, wm[k], ws[k]);
    st->fval[p0 + blockIdx.x] = (s > 0.0) ? m + log(s) : -INFINITY;
  }
}

// f at the current pose from fval[0]; appended to the history.
__global__ void d2d_take_f_kernel(State *st, double *hist, int hist_len) {
  if (threadIdx.x != 0) return;
  st->f = st->fval[0];
  if (!isfinite(st->f)) {
    set_status(&st->status, kStNonFinite);
    st->stopped = 1;
  }
  if (hist && st->hist_n < hist_len) hist[st->hist_n] = st->f;
  st->hist_n++;
}

// Statistics pass at the current pose: per source component i the 27 sums
// of gamma_ij (H entries and gradient) into rows[i].
__global__ __launch_bounds__(kThreads) void d2d_stats_kernel(
    Mix src, Mix tgt, State *st, double *__restrict__ rows) {
  if (st->stopped) return;
  __shared__ double wsum[kWaves][kNStat];
  const int i = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  SrcTerms s;
  src_terms(st->pose[0], src.mu + 3 * i, src.cov + 6 * i, &s);
  const double lwi = src.lw[i];
  const double f = st->f;
  const double *Sp = s.Sp;
  const double SP[9] = {Sp[0], Sp[1], Sp[3], Sp[1], Sp[2], Sp[4], Sp[3], Sp[4], Sp[5]};
  const double *a = s.a;
  double acc[kNStat];
#pragma unroll
  for (int k = 0; k < kNStat; ++k) acc[k] = 0.0;
  for (int j = tid; j < tgt.n; j += kThreads) {
    PairTerms q;
    if (!pair_terms(s, lwi, tgt.mu + 3 * j, tgt.cov + 6 * j, tgt.lw[j], &q)) continue;
    const double gm = exp(q.ell - f);
    const double *L = q.L;
    // g = S^-1 d = L^-T z; P = L^-1; B = S^-1 = P^T P
    double g[3];
    g[2] = q.z[2] / L[5];
    g[1] = (q.z[1] - L[4] * g[2]) / L[2];
    g[0] = (q.z[0] - L[1] * g[1] - L[3] * g[2]) / L[0];
    const double p00 = 1.0 / L[0], p11 = 1.0 / L[2], p22 = 1.0 / L[5];
    const double p10 = -L[1] * p00 / L[2];
    const double p21 = -L[4] * p11 / L[5];
    const double p20 = -(L[3] * p00 + L[4] * p10) / L[5];
    double B[9];
    B[0] = p00 * p00 + p10 * p10 + p20 * p20;
    B[1] = p10 * p11 + p20 * p21;
    B[2] = p20 * p22;
    B[4] = p11 * p11 + p21 * p21;
    B[5] = p21 * p22;
    B[8] = p22 * p22;
    B[3] = B[1]; B[6] = B[2]; B[7] = B[5];
    // gradient in delta: g x a + (A12, A20, A01), A = Sigma' Mm - Mm Sigma',
    // Mm = g g^T - B
    double Mm[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Mm[3 * r + c] = g[r] * g[c] - B[3 * r + c];
    auto Aent = [&](int r, int c) {
      double v = 0.0;
      for (int k = 0; k < 3; ++k) v += SP[3 * r + k] * Mm[3 * k + c] - Mm[3 * r + k] * SP[3 * k + c];
      return v;
    };
    const double gd0 = g[1] * a[2] - g[2] * a[1] + Aent(1, 2);
    const double gd1 = g[2] * a[0] - g[0] * a[2] + Aent(2, 0);
    const double gd2 = g[0] * a[1] - g[1] * a[0] + Aent(0, 1);
    // Gauss-Newton blocks: C = [a]_x B, H_dd = C [a]_x^T, H_dt = C, H_tt = B
    const double ax[9] = {0.0, -a[2], a[1], a[2], 0.0, -a[0], -a[1], a[0], 0.0};
    double C[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        C[3 * r + c] = ax[3 * r] * B[c] + ax[3 * r + 1] * B[3 + c] + ax[3 * r + 2] * B[6 + c];
    // H_dd lower triangle: (C ax^T)_rc = sum_k C_rk ax_ck
    const int ij[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int r = ij[e][0], c = ij[e][1];
      acc[e] += gm * (C[3 * r] * ax[3 * c] + C[3 * r + 1] * ax[3 * c + 1] +
                      C[3 * r + 2] * ax[3 * c + 2]);
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) acc[6 + e] += gm * C[e];
#pragma unroll
    for (int e = 0; e < 6; ++e) acc[15 + e] += gm * B[3 * ij[e][0] + ij[e][1]];
    acc[21] += gm * gd0;
    acc[22] += gm * gd1;
    acc[23] += gm * gd2;
    acc[24] -= gm * g[0];
    acc[25] -= gm * g[1];
    acc[26] -= gm * g[2];
  }
#pragma unroll
  for (int k = 0; k < kNStat; ++k)
    for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
  if (lane == 0)
    for (int k = 0; k < kNStat; ++k) wsum[wv][k] = acc[k];
  __syncthreads();
  if (tid < kNStat) {
    double v = wsum[0][tid];
    for (int k = 1; k < kWaves; ++k) v += wsum[k][tid];
    rows[(size_t)i * kNStat + tid] = v;
  }
}

// Sum of the M statistics rows: thread (g, k) adds column k of the rows
// g, g + G, ... (G = kStepGroups, 16 loads in flight), then thread k the G
// group sums in order.  Then thread 0: the gradient into the state (and,
// when out7 is given, f and df/d(omega, t) for the pose (omega, t) at
// pose6), or the step: Cholesky of H, x = H^-1 grad, the trial poses; the
// stage stops when H is not positive definite or max |x| < kStepTol.
constexpr int kStepGroups = 37;
constexpr int kStepThreads = 1024;   // >= kNStat * kStepGroups

__global__ __launch_bounds__(kStepThreads) void d2d_step_kernel(
    State *st, const double *__restrict__ rows, int M, const double *pose6,
    double *out7) {
  if (st->stopped) return;
  __shared__ double part[kStepGroups][kNStat];
  __shared__ double tot[kNStat];
  const int tid = threadIdx.x;
  if (tid < kNStat * kStepGroups) {
    const int g = tid / kNStat, k = tid - g * kNStat;
    double v = 0.0;
    for (int i = g; i < M; i += 16 * kStepGroups) {
      double u[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = i + e * kStepGroups;
        u[e] = r < M ? rows[(size_t)r * kNStat + k] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) v += u[e];
    }
    part[g][k] = v;
  }
  __syncthreads();
  if (tid < kNStat) {
    double v = part[0][tid];
    for (int g = 1; g < kStepGroups; ++g) v += part[g][tid];
    tot[tid] = v;
  }
  __syncthreads();
  if (tid != 0) return;
  for (int k = 0; k < 6; ++k) st->grad[k] = tot[21 + k];
  if (out7) {
    double J[9];
    left_jacobian(pose6, J);
    out7[0] = st->f;
    for (int c = 0; c < 3; ++c)
      out7[1 + c] = J[c] * tot[21] + J[3 + c] * tot[22] + J[6 + c] * tot[23];
    for (int c = 0; c < 3; ++c) out7[4 + c] = tot[24 + c];
    return;
  }
  // full 6 x 6 H from the blocks (delta first, then t)
  double H[6][6];
  const int ij[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
  for (int e = 0; e < 6; ++e) {
    const int r = ij[e][0], c = ij[e][1];
    H[r][c] = H[c][r] = tot[e];
    H[3 + r][3 + c] = H[3 + c][3 + r] = tot[15 + e];
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) H[r][3 + c] = H[3 + c][r] = tot[6 + 3 * r + c];
  // Cholesky H = L L^T
  double L[6][6] = {};
  for (int j = 0; j < 6; ++j) {
    double s = H[j][j];
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    if (!(s > 0.0) || !isfinite(s)) {
      st->stopped = 1;
      return;
    }
    L[j][j] = sqrt(s);
    for (int i2 = j + 1; i2 < 6; ++i2) {
      double t = H[i2][j];
      for (int k = 0; k < j; ++k) t -= L[i2][k] * L[j][k];
      L[i2][j] = t / L[j][j];
    }
  }
  double y[6], x[6];
  for (int r = 0; r < 6; ++r) {
    double t = st->grad[r];
    for (int k = 0; k < r; ++k) t -= L[r][k] * y[k];
    y[r] = t / L[r][r];
  }
  for (int r = 5; r >= 0; --r) {
    double t = y[r];
    for (int k = r + 1; k < 6; ++k) t -= L[k][r] * x[k];
    x[r] = t / L[r][r];
  }
  double xm = 0.0;
  for (int k = 0; k < 6; ++k) xm = fmax(xm, fabs(x[k]));
  if (!(xm >= kStepTol)) {
    st->stopped = 1;
    return;
  }
  const double *P = st->pose[0];
  for (int k = 0; k < kTrials; ++k) {
    const double sc = ldexp(1.0, -k);
    const double wv3[3] = {sc * x[0], sc * x[1], sc * x[2]};
    double E[9];
    expso3(wv3, E);
    double *Q = st->pose[1 + k];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c)
        Q[3 * r + c] = E[3 * r] * P[c] + E[3 * r + 1] * P[3 + c] + E[3 * r + 2] * P[6 + c];
      Q[9 + r] = P[9 + r] + sc * x[3 + r];
    }
  }
}

// The first trial that increases f becomes the current pose; none: the
// stage ends.
__global__ void d2d_accept_kernel(State *st, double *hist, int hist_len) {
  if (threadIdx.x != 0 || st->stopped) return;
  for (int k = 0; k < kTrials; ++k) {
    if (st->fval[1 + k] > st->f) {
      for (int e = 0; e < kPose; ++e) st->pose[0][e] = st->pose[1 + k][e];
      st->f = st->fval[1 + k];
      st->count[st->stage]++;
      if (hist && st->hist_n < hist_len) hist[st->hist_n] = st->f;
      st->hist_n++;
      return;
    }
  }
  st->stopped = 1;
}

// The current pose as a 4 x 4 transform, the per-stage counts.
__global__ void d2d_out_kernel(const State *st, double *T, int *counts) {
  if (threadIdx.x != 0) return;
  const double *p = st->pose[0];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) T[4 * r + c] = p[3 * r + c];
    T[4 * r + 3] = p[9 + r];
  }
  T[12] = T[13] = T[14] = 0.0;
  T[15] = 1.0;
  if (counts) {
    counts[0] = st->count[0];
    counts[1] = st->count[1];
  }
}

}  // namespace d2d_dev
