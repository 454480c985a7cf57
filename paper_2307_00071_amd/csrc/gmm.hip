// MI355X (gfx950) Gaussian-mixture EM: kernels and the C ABI of include/gmm.h.
//
// One EM iteration is three launches:
//   em_tile_kernel  - persistent tiles of T points.  E-phase: lanes = points,
//                     components wave-uniform (scalar loads of the parameter
//                     block); l_nb (eq. 2-3, in log2 units) goes to LDS, then
//                     a max-shifted log-sum-exp per point (eq. 1-2).
//                     M-phase: lanes = (component, point subset), each lane
//                     reads gamma_nb from LDS and keeps its own sum g, sum g d,
//                     sum g d d^T in registers (FP32 per tile, FP64 across
//                     tiles), so no cross-lane reduction runs per point.  One
//                     FP64 partial row per block.
//   reduce_cols_kernel - fixed-order FP64 sum of the block partials.
//   update_kernel   - FP64 M-step, FP64 3x3 Cholesky, precision Cholesky and
//                     log-normaliser of eq. 3 for the next E-step.
// Every reduction has a fixed order, so a fit is bitwise reproducible for a
// given launch configuration.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "gmm.h"

namespace {

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
enum UpdMode { kUpdFull = 0, kUpdMeanOnly = 1 };

// ------------------------------------------------------------------ layout
// E-step parameter block, per component (16 floats):
//   [0..2] mu  [3] c * log2(e)  [4..9] s * P (P00 P10 P11 P20 P21 P22)
// with s = sqrt(log2(e) / 2), so c' - |P' (x - mu)|^2 = log2(e) * l_nb.
// FP64 state, per component (16 doubles):
//   [0] pi  [1..3] mu  [4..9] Sigma lower (00 10 11 20 21 22)  [10] N_b

// ------------------------------------------------------- device helpers

__device__ inline void set_status(uint32_t *st, uint32_t bits) {
  atomicOr(st, bits);
}

// Cholesky of the 3x3 SPD matrix with lower triangle C = (00 10 11 20 21 22).
// Returns false on a non-positive or non-finite pivot.
__device__ bool chol3(const double *C, double *L) {
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
__device__ void tri_inv3(const double *L, double *P) {
  double p00 = 1.0 / L[0], p11 = 1.0 / L[2], p22 = 1.0 / L[5];
  double p10 = -L[1] * p00 / L[2];
  double p21 = -L[4] * p11 / L[5];
  double p20 = -(L[3] * p00 + L[4] * p10) / L[5];
  P[0] = p00; P[1] = p10; P[2] = p11; P[3] = p20; P[4] = p21; P[5] = p22;
}

// Writes the E-step block and FP64 state of one component from
// (pi, mu, Sigma) in FP64; returns false when Sigma is not SPD.
__device__ bool write_component(int b, double pi, const double *mu,
                                const double *C, double Nb, float *cpar,
                                float4 *shift, double *th64) {
  double *t = th64 + (size_t)b * kTh64Stride;
  t[0] = pi;
  for (int j = 0; j < 3; ++j) t[1 + j] = mu[j];
  for (int j = 0; j < 6; ++j) t[4 + j] = C[j];
  t[10] = Nb;
  float mf0 = (float)mu[0], mf1 = (float)mu[1], mf2 = (float)mu[2];
  shift[b] = make_float4(mf0, mf1, mf2, 0.0f);
  double L[6], P[6];
  bool ok = chol3(C, L);
  float *q = cpar + (size_t)b * kParStride;
  q[0] = mf0; q[1] = mf1; q[2] = mf2;
  if (!ok) {
    // an unusable component: contributes exp2(-inf) = 0 everywhere
    q[3] = -INFINITY;
    for (int j = 0; j < 6; ++j) q[4 + j] = 0.0f;
    return false;
  }
  tri_inv3(L, P);
  double logdiag = log(P[0]) + log(P[2]) + log(P[5]);
  double c = log(pi) - 1.5 * kLn2Pi + logdiag;
  const double s = sqrt(0.5 * kLog2e);
  q[3] = (float)(c * kLog2e);
  for (int j = 0; j < 6; ++j) q[4 + j] = (float)(s * P[j]);
  return true;
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

// ------------------------------------------------------ precompute kernel
// theta_0 given by the caller (FP32 w, mu, cov): FP64 Cholesky of each
// covariance and the eq. 3 terms, weights used as given.
__global__ void precompute_kernel(const float *__restrict__ w,
                                  const float *__restrict__ mu,
                                  const float *__restrict__ cov, int K,
                                  float *cpar, float4 *shift, double *th64,
                                  uint32_t *status) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < K;
       b += gridDim.x * blockDim.x) {
    double pi = w[b];
    double m[3] = {mu[3 * b], mu[3 * b + 1], mu[3 * b + 2]};
    const float *c = cov + 9 * b;
    double C[6] = {c[0], c[3], c[4], c[6], c[7], c[8]};
    if (!(pi > 0.0) || !isfinite(pi) || !isfinite(m[0]) || !isfinite(m[1]) ||
        !isfinite(m[2])) {
      set_status(status, kStBadArg);
      pi = 1.0;
    }
    if (!write_component(b, pi, m, C, 0.0, cpar, shift, th64))
      set_status(status, kStNotSpd);
  }
}

// ------------------------------------------------------------ tile kernel

template <int BLOCK, int T>
struct TileShape {
  static constexpr int G = BLOCK / T;  // component groups in the E-phase
  static constexpr int TS = T + 1;     // padded LDS row (odd: conflict-free)
  static_assert(BLOCK % T == 0, "tile must divide the block");
  static_assert(T % 64 == 0, "a wave must hold one component group");
};

// LDS bytes: [E: max(K*TS floats, BLOCK*10 doubles)][Xs: T float4]
//            [red: 2*G*T floats][wL: BLOCK/64 doubles]
template <int BLOCK, int T>
__host__ __device__ constexpr size_t tile_lds_bytes_e(int K) {
  size_t e = (size_t)K * TileShape<BLOCK, T>::TS * sizeof(float);
  size_t d = (size_t)BLOCK * kNStat * sizeof(double);
  size_t m = e > d ? e : d;
  return (m + 15) & ~(size_t)15;
}

template <int BLOCK, int T>
__host__ __device__ constexpr size_t tile_lds_bytes(int K) {
  return tile_lds_bytes_e<BLOCK, T>(K) + T * sizeof(float4) +
         2 * TileShape<BLOCK, T>::G * T * sizeof(float) +
         (BLOCK / 64) * sizeof(double);
}

// part row layout (ncols = 10 K + 1): stat s of component b at s*K + b; the
// block's sum of lse_n (nats) at 10 K.
template <int BLOCK, int T>
__global__ __launch_bounds__(BLOCK) void em_tile_kernel(
    const float4 *__restrict__ pts, int ntiles, const float *__restrict__ cpar,
    const float4 *__restrict__ shift, int K, int P, int mode,
    double *__restrict__ part, int ncols, float *__restrict__ lse_out) {
  using S = TileShape<BLOCK, T>;
  constexpr int G = S::G, TS = S::TS;
  extern __shared__ __align__(16) unsigned char smem[];
  float *E = reinterpret_cast<float *>(smem);
  unsigned char *p1 = smem + tile_lds_bytes_e<BLOCK, T>(K);
  float4 *Xs = reinterpret_cast<float4 *>(p1);
  float *redm = reinterpret_cast<float *>(p1 + T * sizeof(float4));
  float *reds = redm + G * T;
  double *wL = reinterpret_cast<double *>(reds + G * T);

  const int tid = threadIdx.x;
  const int p = tid % T;
  // T is a multiple of the wave size, so g is wave-uniform; readfirstlane
  // makes that visible to the compiler and the component loop below runs on
  // scalar registers with scalar loads of the parameter block.
  const int g = __builtin_amdgcn_readfirstlane(tid / T);
  const int b_lo = (g * K) / G;
  const int b_hi = ((g + 1) * K) / G;
  const bool mact = tid < K * P;
  const int mb = mact ? tid % K : 0;
  const int mq = mact ? tid / K : 0;
  const float4 sh = shift[mb];
  double acc[kNStat];
#pragma unroll
  for (int j = 0; j < kNStat; ++j) acc[j] = 0.0;
  double Lacc = 0.0;

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const float4 x = pts[(size_t)tile * T + p];
    const int tag = __float_as_int(x.w);
    const bool valid = tag >= 0;
    if (mode != kLabels) {
      float mx = -INFINITY;
      for (int b = b_lo; b < b_hi; ++b) {
        const float *q = cpar + (size_t)b * kParStride;
        float d0 = x.x - q[0], d1 = x.y - q[1], d2 = x.z - q[2];
        float z0 = q[4] * d0;
        float z1 = fmaf(q[5], d0, q[6] * d1);
        float z2 = fmaf(q[7], d0, fmaf(q[8], d1, q[9] * d2));
        float l = fmaf(-z0, z0, q[3]);
        l = fmaf(-z1, z1, l);
        l = fmaf(-z2, z2, l);
        E[b * TS + p] = l;
        mx = fmaxf(mx, l);
      }
      redm[g * T + p] = mx;
      __syncthreads();
      float m = redm[p];
#pragma unroll
      for (int j = 1; j < G; ++j) m = fmaxf(m, redm[j * T + p]);
      float s = 0.0f;
      for (int b = b_lo; b < b_hi; ++b) {
        float e = __builtin_amdgcn_exp2f(E[b * TS + p] - m);
        E[b * TS + p] = e;
        s += e;
      }
      reds[g * T + p] = s;
      __syncthreads();
      if (g == 0) {
        float st = reds[p];
#pragma unroll
        for (int j = 1; j < G; ++j) st += reds[j * T + p];
        float r = valid ? 1.0f / st : 0.0f;
        Xs[p] = make_float4(x.x, x.y, x.z, r);
        if (valid) {
          double lse = ((double)m + (double)log2f(st)) * kLn2;
          Lacc += lse;
          if (lse_out) lse_out[(size_t)tile * T + p] = (float)lse;
        }
      }
    } else {
      for (int b = b_lo; b < b_hi; ++b) E[b * TS + p] = (b == tag) ? 1.0f : 0.0f;
      if (g == 0) Xs[p] = make_float4(x.x, x.y, x.z, valid ? 1.0f : 0.0f);
    }
    __syncthreads();
    if (mode != kSoftLogLik && mact) {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f, a5 = 0.f,
            a6 = 0.f, a7 = 0.f, a8 = 0.f, a9 = 0.f;
      for (int n = mq; n < T; n += P) {
        const float4 xr = Xs[n];
        const float gm = E[mb * TS + n] * xr.w;
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
    __syncthreads();
  }

  double *row = part + (size_t)blockIdx.x * ncols;
  if (mode != kSoftLogLik) {
    double *D = reinterpret_cast<double *>(smem);  // P x 10 x K
    if (mact) {
#pragma unroll
      for (int j = 0; j < kNStat; ++j) D[((size_t)mq * kNStat + j) * K + mb] = acc[j];
    }
    __syncthreads();
    for (int c = tid; c < kNStat * K; c += BLOCK) {
      double s = 0.0;
      for (int q = 0; q < P; ++q) s += D[(size_t)q * kNStat * K + c];
      row[c] = s;
    }
  }
  // block sum of the per-point log-normalisers (fixed butterfly order)
  double v = Lacc;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((tid & 63) == 0) wL[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int j = 0; j < BLOCK / 64; ++j) s += wL[j];
    row[kNStat * K] = s;
  }
}

// ------------------------------------------------------------ reduce kernel
// red[col0 + c] = sum over slots of part[slot][col0 + c], fixed order:
// 16 waves split the slots, then the 16 wave sums are added in wave order.
constexpr int kRedWaves = 16;
__global__ __launch_bounds__(64 * kRedWaves) void reduce_cols_kernel(
    const double *__restrict__ part, int nslots, int ncols, int col0,
    int col1, double *__restrict__ red) {
  __shared__ double sh[kRedWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = col0 + blockIdx.x * 64 + lane;
  double s = 0.0;
  if (col < col1)
    for (int slot = wv; slot < nslots; slot += kRedWaves)
      s += part[(size_t)slot * ncols + col];
  sh[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && col < col1) {
    double t = 0.0;
    for (int j = 0; j < kRedWaves; ++j) t += sh[j][lane];
    red[col] = t;
  }
}

// ------------------------------------------------------------ update kernel
// M-step from the reduced statistics (FP64).  With shift m (the FP32 means
// the tile kernel subtracted) and N0 = sum g, S1 = sum g (x - m),
// S2 = sum g (x - m)(x - m)^T:
//   N_b = N0 + eps,  mu = (S1 + N0 m) / N_b,  delta = mu - m,
//   Sigma = (S2 - S1 delta^T - delta S1^T + N0 delta delta^T) / N_b + lambda I
// which equals sum g (x - mu)(x - mu)^T / N_b + lambda I exactly.
constexpr int kUpdThreads = 1024;
__global__ __launch_bounds__(kUpdThreads) void update_kernel(
    const double *__restrict__ red, int K, double reg, int umode,
    float4 *shift, float *cpar, double *th64, double *loglik_slot,
    uint32_t *status) {
  __shared__ double sN[kUpdThreads];
  const int tid = threadIdx.x;
  // pass 1: new means / covariances and N_b per component
  double Nsum = 0.0;
  for (int b = tid; b < K; b += kUpdThreads) {
    double N0 = red[b];
    double S1[3] = {red[1 * K + b], red[2 * K + b], red[3 * K + b]};
    double S2[6];
    for (int j = 0; j < 6; ++j) S2[j] = red[(4 + j) * K + b];
    float4 mf = shift[b];
    double m[3] = {mf.x, mf.y, mf.z};
    double Nb = N0 + kEpsN;
    double mu[3], dl[3];
    for (int j = 0; j < 3; ++j) {
      mu[j] = (S1[j] + N0 * m[j]) / Nb;
      dl[j] = mu[j] - m[j];
    }
    bool fin = isfinite(N0) && isfinite(S1[0]) && isfinite(S1[1]) && isfinite(S1[2]);
    double *t = th64 + (size_t)b * kTh64Stride;
    if (umode == kUpdMeanOnly) {
      // the next pass accumulates about this mean
      shift[b] = make_float4((float)mu[0], (float)mu[1], (float)mu[2], 0.0f);
      if (!fin) set_status(status, kStNonFinite);
      continue;
    }
    const int ij[6][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
    double C[6];
    for (int j = 0; j < 6; ++j) {
      int r = ij[j][0], c = ij[j][1];
      double v = S2[j] - S1[r] * dl[c] - dl[r] * S1[c] + N0 * dl[r] * dl[c];
      C[j] = v / Nb + ((r == c) ? reg : 0.0);
      fin = fin && isfinite(S2[j]);
    }
    if (!fin) set_status(status, kStNonFinite);
    for (int j = 0; j < 3; ++j) t[1 + j] = mu[j];
    for (int j = 0; j < 6; ++j) t[4 + j] = C[j];
    t[10] = Nb;
  }
  if (tid == 0 && loglik_slot) {
    double L = red[kNStat * K];
    loglik_slot[0] = L;
    if (!isfinite(L)) set_status(status, kStNonFinite);
  }
  if (umode == kUpdMeanOnly) return;
  __syncthreads();
  // pass 2: sum_a N_a (fixed pairwise tree), weights, Cholesky, eq. 3 terms
  for (int b = tid; b < K; b += kUpdThreads) Nsum += th64[(size_t)b * kTh64Stride + 10];
  sN[tid] = Nsum;
  __syncthreads();
  for (int h = kUpdThreads / 2; h > 0; h >>= 1) {
    if (tid < h) sN[tid] += sN[tid + h];
    __syncthreads();
  }
  const double Ntot = sN[0];
  for (int b = tid; b < K; b += kUpdThreads) {
    double *t = th64 + (size_t)b * kTh64Stride;
    double pi = t[10] / Ntot;
    double mu[3] = {t[1], t[2], t[3]};
    double C[6] = {t[4], t[5], t[6], t[7], t[8], t[9]};
    if (!write_component(b, pi, mu, C, t[10], cpar, shift, th64))
      set_status(status, kStNotSpd);
  }
}

// ------------------------------------------------------------ output kernel
// theta (FP64 state) -> caller's FP32 w, mu, full symmetric cov; optionally
// the final log-likelihood from the reduced column.
__global__ void output_kernel(const double *__restrict__ th64, int K, float *w,
                              float *mu, float *cov,
                              const double *__restrict__ red_L,
                              double *loglik_slot, uint32_t *status) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0 && loglik_slot) {
    loglik_slot[0] = red_L[0];
    if (!isfinite(red_L[0])) set_status(status, kStNonFinite);
  }
  if (b >= K) return;
  const double *t = th64 + (size_t)b * kTh64Stride;
  w[b] = (float)t[0];
  for (int j = 0; j < 3; ++j) mu[3 * b + j] = (float)t[1 + j];
  float *c = cov + 9 * b;
  c[0] = (float)t[4];
  c[1] = c[3] = (float)t[5];
  c[4] = (float)t[6];
  c[2] = c[6] = (float)t[7];
  c[5] = c[7] = (float)t[8];
  c[8] = (float)t[9];
}

// ======================================================================= host

thread_local char g_err[512];

gmm_status fail(gmm_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

#define HIP_TRY(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(GMM_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_));   \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Per-thread kernel timing (gmm_profile_*): event pairs around the E+M
// statistics launches, resolved at read time.
struct Profiler {
  bool on = false;
  struct Pair { hipEvent_t a, b; };
  Pair *pairs = nullptr;
  int n = 0, cap = 0;
  ~Profiler() { reset(); free(pairs); }
  void reset() {
    for (int i = 0; i < n; ++i) {
      (void)hipEventDestroy(pairs[i].a);
      (void)hipEventDestroy(pairs[i].b);
    }
    n = 0;
  }
  Pair *next() {
    if (n == cap) {
      int nc = cap ? 2 * cap : 256;
      Pair *np = static_cast<Pair *>(realloc(pairs, sizeof(Pair) * nc));
      if (!np) return nullptr;
      pairs = np;
      cap = nc;
    }
    Pair *p = &pairs[n];
    if (hipEventCreate(&p->a) != hipSuccess) return nullptr;
    if (hipEventCreate(&p->b) != hipSuccess) {
      (void)hipEventDestroy(p->a);
      return nullptr;
    }
    ++n;
    return p;
  }
};
thread_local Profiler g_prof;

struct DevInfo {
  int cus = 0;
  size_t lds_max = 0;
};

DevInfo dev_info() {
  static std::mutex mu;
  static DevInfo cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DevInfo{};
  std::lock_guard<std::mutex> lk(mu);
  if (cache[dev].cus == 0) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) == hipSuccess) {
      cache[dev].cus = pr.multiProcessorCount;
      cache[dev].lds_max = pr.sharedMemPerBlock;
    }
  }
  return cache[dev];
}

// A launch configuration of the tile kernel.
struct TileCfg {
  int block = 0, tile = 0, grid = 0, P = 0;
  size_t lds = 0;
  const void *fn = nullptr;
  void (*launch)(const TileCfg &, hipStream_t, const float4 *, int,
                 const float *, const float4 *, int, int, double *, int,
                 float *) = nullptr;
};

template <int BLOCK, int T>
void launch_tile(const TileCfg &c, hipStream_t s, const float4 *pts, int ntiles,
                 const float *cpar, const float4 *shift, int K, int mode,
                 double *part, int ncols, float *lse) {
  hipLaunchKernelGGL((em_tile_kernel<BLOCK, T>), dim3(c.grid), dim3(BLOCK),
                     c.lds, s, pts, ntiles, cpar, shift, K, c.P, mode, part,
                     ncols, lse);
}

template <int BLOCK, int T>
bool make_cfg(int K, int64_t n, TileCfg *out) {
  DevInfo di = dev_info();
  if (di.cus <= 0) return false;
  if (K > BLOCK) return false;
  size_t lds = tile_lds_bytes<BLOCK, T>(K);
  size_t lds_cap = di.lds_max ? di.lds_max : 65536;
  if (lds > lds_cap) return false;
  const void *fn = reinterpret_cast<const void *>(&em_tile_kernel<BLOCK, T>);
  if (lds > 65536) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
      return false;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BLOCK, lds) !=
          hipSuccess ||
      per_cu <= 0)
    return false;
  int64_t ntiles = (n + T - 1) / T;
  int64_t grid = std::min<int64_t>(ntiles, (int64_t)di.cus * per_cu);
  out->block = BLOCK;
  out->tile = T;
  out->grid = (int)grid;
  out->P = BLOCK / K;
  out->lds = lds;
  out->fn = fn;
  out->launch = &launch_tile<BLOCK, T>;
  return true;
}

bool pick_cfg(int K, int64_t n, TileCfg *out) {
  if (K <= 128 && make_cfg<512, 64>(K, n, out)) return true;
  if (K <= 256 && make_cfg<256, 64>(K, n, out)) return true;
  if (K <= 512 && make_cfg<512, 64>(K, n, out)) return true;
  if (K <= 1024 && make_cfg<1024, 64>(K, n, out)) return true;
  return false;
}

// Workspace layout.
struct WsLayout {
  size_t status, pose64, rt32, cpar, shift, th64, red, part, pts4, total;
  int64_t npad;
  int ncols, nslots;
};

WsLayout ws_layout(int64_t n, int K, const TileCfg &c) {
  WsLayout L{};
  size_t o = 0;
  L.ncols = kNStat * K + 1;
  L.nslots = c.grid;
  L.npad = ((n + c.tile - 1) / c.tile) * c.tile;
  L.status = o; o = align256(o + 256);
  L.pose64 = o; o = align256(o + 32 * sizeof(double));
  L.rt32 = o; o = align256(o + 16 * sizeof(float));
  L.cpar = o; o = align256(o + (size_t)K * kParStride * sizeof(float));
  L.shift = o; o = align256(o + (size_t)K * sizeof(float4));
  L.th64 = o; o = align256(o + (size_t)K * kTh64Stride * sizeof(double));
  L.red = o; o = align256(o + (size_t)L.ncols * sizeof(double));
  L.part = o; o = align256(o + (size_t)L.nslots * L.ncols * sizeof(double));
  L.pts4 = o; o = align256(o + (size_t)L.npad * sizeof(float4));
  L.total = o;
  return L;
}

template <typename T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<unsigned char *>(ws) + off);
}

gmm_status status_from_bits(uint32_t bits) {
  if (bits & kStBadArg) return fail(GMM_ERR_INVALID_ARG, "device: invalid label or parameter");
  if (bits & kStNotSpd) return fail(GMM_ERR_NOT_SPD, "device: covariance not SPD");
  if (bits & kStNonFinite) return fail(GMM_ERR_NONFINITE, "device: non-finite value");
  return GMM_OK;
}

// Owns a stream-ordered workspace when the caller passes none.
struct WsGuard {
  void *ptr = nullptr;
  hipStream_t s = nullptr;
  ~WsGuard() {
    if (ptr) (void)hipFreeAsync(ptr, s);
  }
};

gmm_status get_ws(void **ws, size_t *ws_bytes, size_t need, hipStream_t s,
                  WsGuard *g) {
  if (*ws == nullptr) {
    void *p = nullptr;
    if (hipMallocAsync(&p, need, s) != hipSuccess)
      return fail(GMM_ERR_OOM, "hipMallocAsync(%zu) failed", need);
    g->ptr = p;
    g->s = s;
    *ws = p;
    *ws_bytes = need;
  }
  if (*ws_bytes < need)
    return fail(GMM_ERR_OOM, "workspace %zu bytes < %zu needed", *ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(*ws) & 255)
    return fail(GMM_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  return GMM_OK;
}

gmm_status check_sizes(int64_t n, int32_t k, bool fit) {
  if (n <= 0 || n > GMM_MAX_N) return fail(GMM_ERR_INVALID_ARG, "n=%lld out of range", (long long)n);
  if (k <= 0) return fail(GMM_ERR_INVALID_ARG, "k=%d must be positive", k);
  if (k > GMM_MAX_K) return fail(GMM_ERR_UNSUPPORTED, "k=%d above GMM_MAX_K", k);
  if (fit && k > n) return fail(GMM_ERR_INVALID_ARG, "k=%d > n=%lld", k, (long long)n);
  return GMM_OK;
}

// Launches: tile kernel over all tiles, then the column reduction.
gmm_status run_pass(const TileCfg &c, const WsLayout &L, void *ws, int K,
                    int mode, float *lse, hipStream_t s) {
  int ntiles = (int)(L.npad / c.tile);
  Profiler::Pair *pp = nullptr;
  if (g_prof.on && mode == kSoftStats) {
    pp = g_prof.next();
    if (!pp) return fail(GMM_ERR_DEVICE, "profiling event allocation failed");
    HIP_TRY(hipEventRecord(pp->a, s));
  }
  c.launch(c, s, at<float4>(ws, L.pts4), ntiles, at<float>(ws, L.cpar),
           at<float4>(ws, L.shift), K, mode, at<double>(ws, L.part), L.ncols,
           lse);
  if (pp) HIP_TRY(hipEventRecord(pp->b, s));
  int col0 = (mode == kSoftLogLik) ? kNStat * K : 0;
  int ncol = L.ncols - col0;
  hipLaunchKernelGGL(reduce_cols_kernel, dim3((ncol + 63) / 64),
                     dim3(64 * kRedWaves), 0, s, at<double>(ws, L.part),
                     L.nslots, L.ncols, col0, L.ncols, at<double>(ws, L.red));
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

gmm_status run_update(const WsLayout &L, void *ws, int K, double reg,
                      int umode, double *loglik_slot, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(1), dim3(kUpdThreads), 0, s,
                     at<double>(ws, L.red), K, reg, umode,
                     at<float4>(ws, L.shift), at<float>(ws, L.cpar),
                     at<double>(ws, L.th64), loglik_slot,
                     at<uint32_t>(ws, L.status));
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

gmm_status stage(const float *pts, int64_t n, const WsLayout &L, void *ws,
                 const int32_t *labels, int K, const float *Rt, hipStream_t s) {
  int64_t nb = (L.npad + 255) / 256;
  hipLaunchKernelGGL(stage_kernel, dim3((unsigned)nb), dim3(256), 0, s, pts, n,
                     L.npad, labels, K, Rt, at<float4>(ws, L.pts4),
                     at<uint32_t>(ws, L.status));
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

const char *gmm_status_string(gmm_status s) {
  switch (s) {
    case GMM_OK: return "ok";
    case GMM_ERR_INVALID_ARG: return "invalid argument";
    case GMM_ERR_NOT_SPD: return "covariance not SPD";
    case GMM_ERR_NONFINITE: return "non-finite value";
    case GMM_ERR_OOM: return "out of memory / workspace too small";
    case GMM_ERR_DEVICE: return "HIP runtime error";
    case GMM_ERR_UNSUPPORTED: return "unsupported size";
  }
  return "unknown status";
}

const char *gmm_last_error(void) { return g_err; }

gmm_status gmm_workspace_status(const void *ws, void *stream) {
  if (!ws) return fail(GMM_ERR_INVALID_ARG, "ws is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t bits = 0;
  HIP_TRY(hipMemcpyAsync(&bits, ws, sizeof bits, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return status_from_bits(bits);
}

size_t gmm_fit_workspace_size(int64_t n, int32_t k, const gmm_fit_opts *opts) {
  (void)opts;
  g_err[0] = 0;
  if (check_sizes(n, k, true) != GMM_OK) return 0;
  TileCfg c;
  if (!pick_cfg(k, n, &c)) return 0;
  return ws_layout(n, k, c).total;
}

gmm_status gmm_fit(const float *pts, int64_t n, int32_t k,
                   const int32_t *init_labels, float *w, float *mu, float *cov,
                   double *loglik, const gmm_fit_opts *opts, void *ws,
                   size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  gmm_status st = check_sizes(n, k, true);
  if (st != GMM_OK) return st;
  if (!pts || !w || !mu || !cov || !opts)
    return fail(GMM_ERR_INVALID_ARG, "NULL pointer argument");
  if (opts->iters < 0) return fail(GMM_ERR_INVALID_ARG, "iters < 0");
  if (!(opts->reg_covar >= 0.0) || !isfinite(opts->reg_covar))
    return fail(GMM_ERR_INVALID_ARG, "reg_covar must be finite and >= 0");
  if (opts->moment_mode != GMM_MOMENTS_SHIFTED &&
      opts->moment_mode != GMM_MOMENTS_TWO_PASS)
    return fail(GMM_ERR_INVALID_ARG, "unknown moment_mode");
  if (opts->flags & ~GMM_FLAG_ASYNC) return fail(GMM_ERR_INVALID_ARG, "unknown flags");
  TileCfg c;
  if (!pick_cfg(k, n, &c)) return fail(GMM_ERR_UNSUPPORTED, "no launch configuration for k=%d", k);
  WsLayout L = ws_layout(n, k, c);
  hipStream_t s = static_cast<hipStream_t>(stream);
  WsGuard guard;
  st = get_ws(&ws, &ws_bytes, L.total, s, &guard);
  if (st != GMM_OK) return st;

  HIP_TRY(hipMemsetAsync(at<uint32_t>(ws, L.status), 0, sizeof(uint32_t), s));
  st = stage(pts, n, L, ws, init_labels, k, nullptr, s);
  if (st != GMM_OK) return st;
  const double reg = opts->reg_covar;
  if (init_labels) {
    // theta_0 = M-step of the one-hot responsibilities, two passes: the mean
    // (shift 0), then the scatter about it.
    HIP_TRY(hipMemsetAsync(at<float4>(ws, L.shift), 0, sizeof(float4) * k, s));
    if ((st = run_pass(c, L, ws, k, kLabels, nullptr, s)) != GMM_OK) return st;
    if ((st = run_update(L, ws, k, reg, kUpdMeanOnly, nullptr, s)) != GMM_OK) return st;
    if ((st = run_pass(c, L, ws, k, kLabels, nullptr, s)) != GMM_OK) return st;
    if ((st = run_update(L, ws, k, reg, kUpdFull, nullptr, s)) != GMM_OK) return st;
  } else {
    int nb = (k + 255) / 256;
    hipLaunchKernelGGL(precompute_kernel, dim3(nb), dim3(256), 0, s, w, mu, cov,
                       k, at<float>(ws, L.cpar), at<float4>(ws, L.shift),
                       at<double>(ws, L.th64), at<uint32_t>(ws, L.status));
    HIP_TRY(hipGetLastError());
  }
  for (int t = 0; t < opts->iters; ++t) {
    double *slot = loglik ? loglik + t : nullptr;
    if (opts->moment_mode == GMM_MOMENTS_TWO_PASS) {
      if ((st = run_pass(c, L, ws, k, kSoftStats, nullptr, s)) != GMM_OK) return st;
      if ((st = run_update(L, ws, k, reg, kUpdMeanOnly, slot, s)) != GMM_OK) return st;
      slot = nullptr;
    }
    if ((st = run_pass(c, L, ws, k, kSoftStats, nullptr, s)) != GMM_OK) return st;
    if ((st = run_update(L, ws, k, reg, kUpdFull, slot, s)) != GMM_OK) return st;
  }
  // log-likelihood of the returned parameters, and the FP32 outputs
  if ((st = run_pass(c, L, ws, k, kSoftLogLik, nullptr, s)) != GMM_OK) return st;
  hipLaunchKernelGGL(output_kernel, dim3((k + 255) / 256), dim3(256), 0, s,
                     at<double>(ws, L.th64), k, w, mu, cov,
                     at<double>(ws, L.red) + kNStat * k,
                     loglik ? loglik + opts->iters : nullptr,
                     at<uint32_t>(ws, L.status));
  HIP_TRY(hipGetLastError());
  if (opts->flags & GMM_FLAG_ASYNC) return GMM_OK;
  uint32_t bits = 0;
  HIP_TRY(hipMemcpyAsync(&bits, at<uint32_t>(ws, L.status), sizeof bits,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return status_from_bits(bits);
}

size_t gmm_loglik_workspace_size(int64_t n, int32_t k) {
  g_err[0] = 0;
  if (check_sizes(n, k, false) != GMM_OK) return 0;
  TileCfg c;
  if (!pick_cfg(k, n, &c)) return 0;
  return ws_layout(n, k, c).total;
}

gmm_status gmm_loglik(const float *pts, int64_t n, const float *pose6,
                      int32_t k, const float *w, const float *mu,
                      const float *cov, double *out_L, float *out_lse,
                      void *ws, size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  gmm_status st = check_sizes(n, k, false);
  if (st != GMM_OK) return st;
  if (!pts || !w || !mu || !cov || !out_L)
    return fail(GMM_ERR_INVALID_ARG, "NULL pointer argument");
  TileCfg c;
  if (!pick_cfg(k, n, &c)) return fail(GMM_ERR_UNSUPPORTED, "no launch configuration for k=%d", k);
  WsLayout L = ws_layout(n, k, c);
  hipStream_t s = static_cast<hipStream_t>(stream);
  WsGuard guard;
  st = get_ws(&ws, &ws_bytes, L.total, s, &guard);
  if (st != GMM_OK) return st;
  HIP_TRY(hipMemsetAsync(at<uint32_t>(ws, L.status), 0, sizeof(uint32_t), s));
  const float *Rt = nullptr;
  if (pose6) {
    hipLaunchKernelGGL(pose_kernel, dim3(1), dim3(64), 0, s, pose6,
                       at<double>(ws, L.pose64), at<float>(ws, L.rt32));
    HIP_TRY(hipGetLastError());
    Rt = at<float>(ws, L.rt32);
  }
  if ((st = stage(pts, n, L, ws, nullptr, k, Rt, s)) != GMM_OK) return st;
  int nb = (k + 255) / 256;
  hipLaunchKernelGGL(precompute_kernel, dim3(nb), dim3(256), 0, s, w, mu, cov,
                     k, at<float>(ws, L.cpar), at<float4>(ws, L.shift),
                     at<double>(ws, L.th64), at<uint32_t>(ws, L.status));
  HIP_TRY(hipGetLastError());
  if ((st = run_pass(c, L, ws, k, kSoftLogLik, out_lse, s)) != GMM_OK) return st;
  HIP_TRY(hipMemcpyAsync(out_L, at<double>(ws, L.red) + kNStat * k,
                         sizeof(double), hipMemcpyDeviceToDevice, s));
  return GMM_OK;
}

gmm_status gmm_profile_enable(int on) {
  g_prof.on = on != 0;
  return GMM_OK;
}

gmm_status gmm_profile_read(double *tile_ms_total, int64_t *tile_launches) {
  double tot = 0.0;
  for (int i = 0; i < g_prof.n; ++i) {
    HIP_TRY(hipEventSynchronize(g_prof.pairs[i].b));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, g_prof.pairs[i].a, g_prof.pairs[i].b));
    tot += ms;
  }
  if (tile_ms_total) *tile_ms_total = tot;
  if (tile_launches) *tile_launches = g_prof.n;
  g_prof.reset();
  return GMM_OK;
}

size_t gmm_loglik_backward_workspace_size(int64_t n, int32_t k) {
  return gmm_loglik_workspace_size(n, k);
}

gmm_status gmm_loglik_backward(const float *pts, int64_t n, const float *pose6,
                               int32_t k, const float *w, const float *mu,
                               const float *cov, const float *lse,
                               const double *grad_L, float *g_pose6,
                               float *g_pts, float *g_w, float *g_mu,
                               float *g_cov, void *ws, size_t ws_bytes,
                               void *stream) {
  (void)pts; (void)n; (void)pose6; (void)k; (void)w; (void)mu; (void)cov;
  (void)lse; (void)grad_L; (void)g_pose6; (void)g_pts; (void)g_w; (void)g_mu;
  (void)g_cov; (void)ws; (void)ws_bytes; (void)stream;
  return fail(GMM_ERR_UNSUPPORTED, "gmm_loglik_backward not built yet");
}

}  // extern "C"
