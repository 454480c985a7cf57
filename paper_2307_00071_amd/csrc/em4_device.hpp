// Device code of the 4D (x, y, z, intensity) mixture: EM tile kernel,
// reduction, FP64 M-step update, conditional intensity and joint sampling.
//
// The paper's model is a mixture over 4D points (Sec. IV "GIRA
// Reconstruction"; Sec. V: weights (1, K, 1), means (1, K, 4), covariances
// (1, K, 4, 4)) fitted by the EM of Sec. V "Expectation Maximization" (eq.
// 1-3 with D = 4).  The kernels follow the 3D dense tile kernel's plan:
// points in lanes for the E-step, (component, point subset) in lanes for the
// M-step statistics, responsibilities only in LDS, FP64 partial rows.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gmm.h"
#include "wave_f64.hpp"

namespace gmm4_dev {

using namespace gmm_wave;

constexpr double kLog2e = 1.44269504088896340736;
constexpr double kLn2 = 0.693147180559945309417;
constexpr double kLn2Pi = 1.83787706640934548356;
constexpr double kEpsN = 10.0 * 2.220446049250313080847e-16;  // N_b guard
constexpr int kPar = 16;    // floats per component in the E-step block
constexpr int kTh = 16;     // doubles per component in the FP64 state
constexpr int kNStat = 15;  // N, S1 (4), S2 lower triangle (10)
constexpr int kBlock = 512;
constexpr int kT = 64;      // points per tile (one wave)
constexpr int kTS = kT + 1; // LDS row stride (odd: conflict-free)
constexpr int kMaxK = 512;
constexpr int kRedChunks = 4;
constexpr int kUpdThreads = 512;

constexpr uint32_t kStBadArg = 1u << GMM_ERR_INVALID_ARG;
constexpr uint32_t kStNotSpd = 1u << GMM_ERR_NOT_SPD;
constexpr uint32_t kStNonFinite = 1u << GMM_ERR_NONFINITE;

enum { kSoftStats = 0, kSoftLogLik = 1, kLabels = 2 };
enum { kUpdFull = 0, kUpdMeanOnly = 1, kUpdNone = 2 };

// Lower triangle of a symmetric 4 x 4 matrix, row by row: (0,0) (1,0)
// (1,1) (2,0) (2,1) (2,2) (3,0) (3,1) (3,2) (3,3).
__host__ __device__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }

__device__ inline void set_status(uint32_t *st, uint32_t bits) {
  atomicOr(st, bits);
}

// Cholesky Sigma = L L^T (lower triangle in, lower factor out) and P = L^-1;
// false when a pivot is not positive and finite.  FP64.
__device__ inline bool chol_inv4(const double *C, double *L, double *P) {
  for (int j = 0; j < 4; ++j) {
    double s = C[tri(j, j)];
    for (int k = 0; k < j; ++k) s -= L[tri(j, k)] * L[tri(j, k)];
    if (!(s > 0.0) || !isfinite(s)) return false;
    const double d = sqrt(s);
    L[tri(j, j)] = d;
    for (int i = j + 1; i < 4; ++i) {
      double t = C[tri(i, j)];
      for (int k = 0; k < j; ++k) t -= L[tri(i, k)] * L[tri(j, k)];
      L[tri(i, j)] = t / d;
    }
  }
  // forward substitution, column by column: P L = I
  for (int c = 0; c < 4; ++c) {
    P[tri(c, c)] = 1.0 / L[tri(c, c)];
    for (int r = c + 1; r < 4; ++r) {
      double t = 0.0;
      for (int k = c; k < r; ++k) t -= L[tri(r, k)] * P[tri(k, c)];
      P[tri(r, c)] = t / L[tri(r, r)];
    }
  }
  return true;
}

// l'_pb of one component: log2(e) (l_pb - C) from the E-step block
// q = (mu (4), c', P' (10 lower)), P' = sqrt(log2(e) / 2) P.
__device__ __forceinline__ float logterm4(const float *__restrict__ q, float4 x) {
  const float d0 = x.x - q[0], d1 = x.y - q[1], d2 = x.z - q[2], d3 = x.w - q[3];
  const float z0 = q[5] * d0;
  const float z1 = fmaf(q[6], d0, q[7] * d1);
  const float z2 = fmaf(q[8], d0, fmaf(q[9], d1, q[10] * d2));
  const float z3 = fmaf(q[11], d0, fmaf(q[12], d1, fmaf(q[13], d2, q[14] * d3)));
  float l = fmaf(-z0, z0, q[4]);
  l = fmaf(-z1, z1, l);
  l = fmaf(-z2, z2, l);
  return fmaf(-z3, z3, l);
}

struct Tile4Args {
  int64_t n;      // points
  int ntiles, K, P, mode, ncols;
  int cmaj = 0;   // partial row component-major (b kNStat + j), for the fused update
};

// LDS: E rows (K x kTS floats), Xs (kTS float4), Rs (kTS floats),
// partial normalisers (G x kT), wL (waves doubles); the end-of-kernel
// subset sums reuse the E rows (P x K doubles).
__host__ __device__ constexpr size_t tile4_lds_bytes(int K) {
  const size_t e = (size_t)K * kTS * sizeof(float);
  const size_t d = (size_t)kBlock * sizeof(double);
  const size_t m = ((e > d ? e : d) + 15) & ~(size_t)15;
  return m + kTS * sizeof(float4) + kTS * sizeof(float) +
         (size_t)(kBlock / kT) * kT * sizeof(float) + kT * sizeof(float) +
         (kBlock / 64) * sizeof(double);
}

// One E+M pass (or an L-only pass) over tiles of kT points, grid-strided.
// Lanes of the E-phase: point p = tid % kT of component group g = tid / kT
// (wave-uniform; the group's components are read with scalar loads).
// Lanes of the M-phase: component mb = tid % K, point subset mq = tid / K
// of TRIP consecutive points (P subsets x TRIP = kT).
template <int TRIP>
__global__ __launch_bounds__(kBlock) void em4_tile_kernel(
    const float4 *__restrict__ pts, const int32_t *__restrict__ labels,
    const float *__restrict__ cpar, const float4 *__restrict__ shift,
    double *__restrict__ part, Tile4Args a) {
  constexpr int G = kBlock / kT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int K = a.K, P = a.P, mode = a.mode;
  float *E = reinterpret_cast<float *>(smem);
  const size_t eb = (((size_t)K * kTS * sizeof(float) > kBlock * sizeof(double)
                          ? (size_t)K * kTS * sizeof(float)
                          : kBlock * sizeof(double)) + 15) & ~(size_t)15;
  float4 *Xs = reinterpret_cast<float4 *>(smem + eb);
  float *Rs = reinterpret_cast<float *>(Xs + kTS);
  float *reds = Rs + kTS;
  float *Mp = reds + G * kT;
  double *wL = reinterpret_cast<double *>(Mp + kT);

  const int tid = threadIdx.x;
  const int p = tid % kT;
  const int g = __builtin_amdgcn_readfirstlane(tid / kT);
  const int b_lo = (g * K) / G, b_hi = ((g + 1) * K) / G;
  const bool mact = tid < K * P;
  const int mb = mact ? tid % K : 0;
  const int mq = mact ? tid / K : 0;
  const double Cb = *reinterpret_cast<const double *>(cpar + (size_t)K * kPar);
  const float4 sh = shift[mb];
  double acc[kNStat];
#pragma unroll
  for (int j = 0; j < kNStat; ++j) acc[j] = 0.0;
  double Lacc = 0.0;

  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int64_t idx = (int64_t)tile * kT + p;
    float4 x = idx < a.n ? pts[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
    // a non-finite point (reported by check4_kernel) takes no part
    const bool valid = idx < a.n && isfinite(x.x) && isfinite(x.y) && isfinite(x.z) &&
                       isfinite(x.w);
    if (!valid) x = make_float4(0.f, 0.f, 0.f, 0.f);
    if (mode != kLabels) {
      float s = 0.0f;
      for (int b = b_lo; b < b_hi; ++b) {
        const float e = __builtin_amdgcn_exp2f(logterm4(cpar + (size_t)b * kPar, x));
        E[b * kTS + p] = e;
        s += e;
      }
      reds[g * kT + p] = s;
      __syncthreads();
      if (g == 0) {
        float st = reds[p];
#pragma unroll
        for (int j = 1; j < G; ++j) st += reds[j * kT + p];
        float mref = 0.0f;
        if (valid && !(st >= 0x1p-100f)) {
          // far from every component: exact max-shifted sum for this point
          float m = -INFINITY;
          for (int bb = 0; bb < K; ++bb) m = fmaxf(m, logterm4(cpar + (size_t)bb * kPar, x));
          st = 0.0f;
          for (int bb = 0; bb < K; ++bb) {
            const float e = __builtin_amdgcn_exp2f(logterm4(cpar + (size_t)bb * kPar, x) - m);
            E[bb * kTS + p] = e;
            st += e;
          }
          mref = m;
        }
        Xs[p] = x;
        Rs[p] = valid ? __builtin_amdgcn_rcpf(st) : 0.0f;
        Mp[p] = mref;
        if (valid) Lacc += (Cb + (double)mref + (double)__builtin_amdgcn_logf(st)) * kLn2;
      }
    } else {
      const int lab = valid ? labels[idx] : -1;
      for (int b = b_lo; b < b_hi; ++b) E[b * kTS + p] = (b == lab) ? 1.0f : 0.0f;
      if (g == 0) {
        Xs[p] = x;
        Rs[p] = valid ? 1.0f : 0.0f;
      }
    }
    __syncthreads();
    if (mode != kSoftLogLik && mact) {
      const float *Eb = E + mb * kTS + mq * TRIP;
      const float4 *Xb = Xs + mq * TRIP;
      const float *Rb = Rs + mq * TRIP;
      float v[kNStat];
#pragma unroll
      for (int j = 0; j < kNStat; ++j) v[j] = 0.0f;
#pragma unroll 4
      for (int j = 0; j < TRIP; ++j) {
        const float4 xr = Xb[j];
        const float gm = Eb[j] * Rb[j];
        const float d[4] = {xr.x - sh.x, xr.y - sh.y, xr.z - sh.z, xr.w - sh.w};
        v[0] += gm;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float wr = gm * d[r];
          v[1 + r] += wr;
#pragma unroll
          for (int c = 0; c <= r; ++c) v[5 + tri(r, c)] = fmaf(wr, d[c], v[5 + tri(r, c)]);
        }
      }
#pragma unroll
      for (int j = 0; j < kNStat; ++j) acc[j] += (double)v[j];
    }
    __syncthreads();
  }

  double *row = part + (size_t)blockIdx.x * a.ncols;
  if (mode != kSoftLogLik) {
    double *Dd = reinterpret_cast<double *>(smem);  // P x K
#pragma unroll
    for (int j = 0; j < kNStat; ++j) {
      __syncthreads();
      if (mact) Dd[mq * K + mb] = acc[j];
      __syncthreads();
      for (int i = tid; i < K; i += kBlock) {
        double sum = 0.0;
        for (int qq = 0; qq < P; ++qq) sum += Dd[qq * K + i];
        row[a.cmaj ? i * kNStat + j : j * K + i] = sum;
      }
    }
  }
  double v = Lacc;
  v = wave_sum_f64(v);
  if ((tid & 63) == 0) wL[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int j = 0; j < kBlock / 64; ++j) sum += wL[j];
    row[kNStat * K] = sum;
  }
}

// red[y][c] = sum of part[r][c] over the rows r of chunk y (in row order).
__global__ __launch_bounds__(256) void reduce4_kernel(const double *__restrict__ part,
                                                      int rows, int ncols,
                                                      double *__restrict__ red) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  if (c >= ncols) return;
  const int r0 = (int)(((int64_t)rows * y) / gridDim.y);
  const int r1 = (int)(((int64_t)rows * (y + 1)) / gridDim.y);
  double s = 0.0;
  for (int r = r0; r < r1; ++r) s += part[(size_t)r * ncols + c];
  red[(size_t)y * ncols + c] = s;
}

// Every point finite (status NONFINITE otherwise) and every label in
// [0, K) (INVALID_ARG otherwise).
__global__ __launch_bounds__(256) void check4_kernel(const float4 *__restrict__ pts,
                                                     const int32_t *__restrict__ labels,
                                                     int64_t n, int K, uint32_t *status) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float4 x = pts[i];
  if (!(isfinite(x.x) && isfinite(x.y) && isfinite(x.z) && isfinite(x.w)))
    set_status(status, kStNonFinite);
  if (labels) {
    const int l = labels[i];
    if (l < 0 || l >= K) set_status(status, kStBadArg);
  }
}

__global__ void init4_kernel(uint32_t *status, float4 *shift, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *status = 0u;
  if (shift)
    for (int b = i; b < K; b += gridDim.x * blockDim.x)
      shift[b] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// The E-step block of one component from mu and P (FP64); returns
// ln(w P00 P11 P22 P33) or -inf when the covariance is not SPD.
__device__ inline double store_block4(float *q, const double *mu, const double *C, double w) {
  double L[10], P[10];
  for (int j = 0; j < 4; ++j) q[j] = (float)mu[j];
  q[15] = 0.0f;
  if (!chol_inv4(C, L, P)) {
    for (int j = 0; j < 10; ++j) q[5 + j] = 0.0f;
    return -INFINITY;
  }
  const double s = sqrt(0.5 * kLog2e);
  for (int j = 0; j < 10; ++j) q[5 + j] = (float)(s * P[j]);
  return log(w * P[tri(0, 0)] * P[tri(1, 1)] * P[tri(2, 2)] * P[tri(3, 3)]);
}

// Block-wide max and sum in a fixed order (NT threads, one value each).
template <int NT>
__device__ inline void block_sum_max(double &sum, double &mx, double *scratch) {
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_xor(sum, off, 64);
    mx = fmax(mx, __shfl_xor(mx, off, 64));
  }
  constexpr int NW = NT / 64;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    scratch[threadIdx.x >> 6] = sum;
    scratch[NW + (threadIdx.x >> 6)] = mx;
  }
  __syncthreads();
  sum = scratch[0];
  mx = scratch[NW];
  for (int j = 1; j < NW; ++j) {
    sum += scratch[j];
    mx = fmax(mx, scratch[NW + j]);
  }
}

struct Upd4Args {
  int K, ncols, mode, umode, chunks;
  double reg;
};

// One block (thread b = component b): the reduced statistics about the
// shift m (columns s*K + b), the M-step
//   N_b = N0 + eps, mu = (S1 + N0 m) / N_b, delta = mu - m,
//   Sigma = (S2 - S1 delta^T - delta S1^T + N0 delta delta^T) / N_b + lambda I,
//   pi_b = N_b / sum_a N_a,
// then the eq. 3 terms of the next E-step with the bound C = max_b c_b
// (c_b - C stored, C in the header).  Also the log-likelihood of the pass
// (column 15 K) and, when asked, the FP32 outputs.
__global__ __launch_bounds__(kUpdThreads) void update4_kernel(
    const double *__restrict__ red, const float *__restrict__ cpar_in,
    const float4 *__restrict__ shift_in, float *__restrict__ cpar_out,
    float4 *__restrict__ shift_out, double *__restrict__ th64,
    double *loglik_slot, float *out_w, float *out_mu, float *out_cov,
    uint32_t *status, Upd4Args a) {
  __shared__ double scratch[2 * kUpdThreads / 64];
  const int K = a.K, b = threadIdx.x;
  const bool act = b < K;
  auto col = [&](int c) {
    double t = 0.0;
    for (int y = 0; y < a.chunks; ++y) t += red[(size_t)y * a.ncols + c];
    return t;
  };
  if (threadIdx.x == 0 && loglik_slot) {
    const double L = col(kNStat * K);
    *loglik_slot = L;
    if (!isfinite(L)) set_status(status, kStNonFinite);
  }
  if (a.umode == kUpdNone) {
    // outputs of the current parameters
    if (act && out_w) {
      const double *t = th64 + (size_t)b * kTh;
      out_w[b] = (float)t[0];
      for (int j = 0; j < 4; ++j) out_mu[4 * b + j] = (float)t[1 + j];
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
          out_cov[16 * b + 4 * r + c] = (float)t[5 + (r >= c ? tri(r, c) : tri(c, r))];
    }
    return;
  }
  if (a.umode == kUpdMeanOnly) {
    if (act) {
      const double N0 = col(b);
      const float4 mf = shift_in[b];
      const double m[4] = {mf.x, mf.y, mf.z, mf.w};
      float mu[4];
      bool fin = isfinite(N0);
      for (int j = 0; j < 4; ++j) {
        const double S1 = col((1 + j) * K + b);
        fin = fin && isfinite(S1);
        mu[j] = (float)((S1 + N0 * m[j]) / (N0 + kEpsN));
      }
      if (!fin) set_status(status, kStNonFinite);
      shift_out[b] = make_float4(mu[0], mu[1], mu[2], mu[3]);
    }
    for (int i = b; i < (K + 1) * kPar; i += kUpdThreads) cpar_out[i] = cpar_in[i];
    return;
  }
  double Nb = 0.0, mu[4] = {0, 0, 0, 0}, C[10];
  for (int j = 0; j < 10; ++j) C[j] = 0.0;
  if (act) {
    const double N0 = col(b);
    double S1[4];
    for (int j = 0; j < 4; ++j) S1[j] = col((1 + j) * K + b);
    const float4 mf = shift_in[b];
    const double m[4] = {mf.x, mf.y, mf.z, mf.w};
    Nb = N0 + kEpsN;
    const double rN = 1.0 / Nb;
    double dl[4];
    bool fin = isfinite(N0);
    for (int j = 0; j < 4; ++j) {
      mu[j] = (S1[j] + N0 * m[j]) * rN;
      dl[j] = mu[j] - m[j];
      fin = fin && isfinite(S1[j]);
    }
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c <= r; ++c) {
        const double s2 = col((5 + tri(r, c)) * K + b);
        const double v = s2 - S1[r] * dl[c] - dl[r] * S1[c] + N0 * dl[r] * dl[c];
        C[tri(r, c)] = v * rN + (r == c ? a.reg : 0.0);
        fin = fin && isfinite(s2);
      }
    if (!fin) set_status(status, kStNonFinite);
  }
  // ln(N_b P00 P11 P22 P33) before the reductions: with pi_b = N_b / N,
  // c_b - max_a c_a = cb - max_a cb_a (ln N cancels)
  float *q = cpar_out + (size_t)b * kPar;
  double cb = -INFINITY;
  if (act) {
    cb = store_block4(q, mu, C, Nb);
    if (!isfinite(cb)) set_status(status, kStNotSpd);
  }
  double sN = act ? Nb : 0.0, mx = cb;
  block_sum_max<kUpdThreads>(sN, mx, scratch);
  if (act) {
    double *t = th64 + (size_t)b * kTh;
    t[0] = Nb / sN;
    for (int j = 0; j < 4; ++j) t[1 + j] = mu[j];
    for (int j = 0; j < 10; ++j) t[5 + j] = C[j];
    t[15] = Nb;
    shift_out[b] = make_float4((float)mu[0], (float)mu[1], (float)mu[2], (float)mu[3]);
    q[4] = isfinite(cb) ? (float)((cb - mx) * kLog2e) : -INFINITY;
  }
  if (b == 0) {
    const double Cmax = isfinite(mx) ? (mx - log(sN) - 2.0 * kLn2Pi) * kLog2e : 0.0;
    *reinterpret_cast<double *>(cpar_out + (size_t)K * kPar) = Cmax;
  }
}

// Fused reduction and M-step for lambda > 0 (one launch per pass instead of
// reduce4_kernel + update4_kernel).  Every eigenvalue of an updated Sigma_b
// is at least lambda, so prod_j P_jj <= lambda^-2 and, with pi_b <= 1,
// c_b <= C + ln K for the static C = -2 ln(lambda) - 2 ln(2 pi) - ln K: the
// stored c_b - C is at most log2 K (no FP32 overflow of a point's sum) and
// near 0 for a typical weight 1/K; sum_a N_a = n + K eps (each point's
// responsibilities sum to one).  So each component is updated on its own:
// block b sums its 15 columns of the component-major partial rows (thread
// (g, s) statistic s of rows g, g + G, ..., 16 loads in flight, then half
// a wave per statistic adds the G group sums: DPP rows, then the two rows
// in order), thread 0 updates it in FP64; the last wave of block 0 sums the
// log-likelihood column.  Bitwise reproducible.
constexpr int kFuse4Groups = 32;   // one per lane of a half wave
constexpr int kFuse4Lwave = (kNStat * kFuse4Groups + 63) / 64 * 64;   // first thread of the L wave
constexpr int kFuse4Threads = kFuse4Lwave + 64;

struct Fuse4Args {
  int K, ncols, nrows, mode, umode;
  double reg;
  double lnZ;    // ln(n + K eps) - 2 ln(lambda) - ln K: c_b - C = ln(N_b prod P_jj) - lnZ
  double Ntot;   // n + K eps
  double Chdr;   // C log2(e)
};

__global__ __launch_bounds__(kFuse4Threads) void reduce_update4_kernel(
    const double *__restrict__ part, const float *__restrict__ cpar_in,
    const float4 *__restrict__ shift_in, float *__restrict__ cpar_out,
    float4 *__restrict__ shift_out, double *__restrict__ th64, double *loglik_slot,
    float *out_w, float *out_mu, float *out_cov, uint32_t *status, Fuse4Args a) {
  __shared__ double sums[kFuse4Groups * kNStat];
  __shared__ double tot[kNStat + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int K = a.K, b = blockIdx.x;
  const bool lcol = b == 0 && a.mode != kLabels;
  const bool stats = a.mode != kSoftLogLik;
  constexpr int NS = kNStat * kFuse4Groups;
  if (tid < NS) {
    if (stats) {
      const int g = tid / kNStat, st = tid - g * kNStat;
      const double *src = part + (size_t)b * kNStat + st;
      constexpr int G = kFuse4Groups;
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
  } else if (tid >= kFuse4Lwave && lcol) {   // one whole wave
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
  // wave w adds the G = 32 group sums of statistics 2w (lanes 0-31) and
  // 2w + 1 (lanes 32-63), lane g of a half holding group g
  __syncthreads();
  if (stats && 2 * (tid >> 6) < kNStat) {
    const int w = tid >> 6, st = 2 * w + (lane >> 5);
    const double2 h = half_sums_f64(st < kNStat ? sums[(lane & 31) * kNStat + st] : 0.0);
    if (lane == 0) tot[2 * w] = h.x;
    if (lane == 0 && 2 * w + 1 < kNStat) tot[2 * w + 1] = h.y;
  }
  __syncthreads();
  if (tid != 0) return;
  if (lcol && loglik_slot) {
    const double L = tot[kNStat];
    *loglik_slot = L;
    if (!isfinite(L)) set_status(status, kStNonFinite);
  }
  if (a.umode == kUpdNone) {
    if (out_w) {
      const double *t = th64 + (size_t)b * kTh;
      out_w[b] = (float)t[0];
      for (int j = 0; j < 4; ++j) out_mu[4 * b + j] = (float)t[1 + j];
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
          out_cov[16 * b + 4 * r + c] = (float)t[5 + (r >= c ? tri(r, c) : tri(c, r))];
    }
    return;
  }
  const double N0 = tot[0];
  double S1[4];
  for (int j = 0; j < 4; ++j) S1[j] = tot[1 + j];
  const float4 mf = shift_in[b];
  const double m[4] = {mf.x, mf.y, mf.z, mf.w};
  const double Nb = N0 + kEpsN;
  const double rN = 1.0 / Nb;
  double mu[4], dl[4];
  bool fin = isfinite(N0);
  for (int j = 0; j < 4; ++j) {
    mu[j] = (S1[j] + N0 * m[j]) * rN;
    dl[j] = mu[j] - m[j];
    fin = fin && isfinite(S1[j]);
  }
  if (a.umode == kUpdMeanOnly) {
    if (!fin) set_status(status, kStNonFinite);
    shift_out[b] = make_float4((float)mu[0], (float)mu[1], (float)mu[2], (float)mu[3]);
    for (int j = 0; j < kPar; ++j) cpar_out[(size_t)b * kPar + j] = cpar_in[(size_t)b * kPar + j];
    if (b == 0)
      *reinterpret_cast<double *>(cpar_out + (size_t)K * kPar) =
          *reinterpret_cast<const double *>(cpar_in + (size_t)K * kPar);
    return;
  }
  double C[10];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c <= r; ++c) {
      const double s2 = tot[5 + tri(r, c)];
      const double v = s2 - S1[r] * dl[c] - dl[r] * S1[c] + N0 * dl[r] * dl[c];
      C[tri(r, c)] = v * rN + (r == c ? a.reg : 0.0);
      fin = fin && isfinite(s2);
    }
  if (!fin) set_status(status, kStNonFinite);
  float *q = cpar_out + (size_t)b * kPar;
  const double cb = store_block4(q, mu, C, Nb);
  if (!isfinite(cb)) set_status(status, kStNotSpd);
  double *t = th64 + (size_t)b * kTh;
  t[0] = Nb / a.Ntot;
  for (int j = 0; j < 4; ++j) t[1 + j] = mu[j];
  for (int j = 0; j < 10; ++j) t[5 + j] = C[j];
  t[15] = Nb;
  shift_out[b] = make_float4((float)mu[0], (float)mu[1], (float)mu[2], (float)mu[3]);
  q[4] = isfinite(cb) ? (float)((cb - a.lnZ) * kLog2e) : -INFINITY;
  if (b == 0) *reinterpret_cast<double *>(cpar_out + (size_t)K * kPar) = a.Chdr;
}

// Caller-supplied parameters (FP32 w, mu K x 4, cov K x 4 x 4) -> FP64 state,
// E-step block and shifts; weights used as given (must be > 0).
__global__ __launch_bounds__(kUpdThreads) void precompute4_kernel(
    const float *__restrict__ w, const float *__restrict__ mu,
    const float *__restrict__ cov, int K, float *__restrict__ cpar,
    float4 *__restrict__ shift, double *__restrict__ th64, uint32_t *status) {
  __shared__ double scratch[2 * kUpdThreads / 64];
  const int b = threadIdx.x;
  const bool act = b < K;
  double cb = -INFINITY;
  float *q = cpar + (size_t)b * kPar;
  if (act) {
    double m[4], C[10];
    for (int j = 0; j < 4; ++j) m[j] = mu[4 * b + j];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c <= r; ++c) C[tri(r, c)] = cov[16 * b + 4 * r + c];
    const double wb = w[b];
    if (!(wb > 0.0) || !isfinite(wb)) set_status(status, kStBadArg);
    cb = store_block4(q, m, C, wb);
    if (!isfinite(cb)) set_status(status, kStNotSpd);
    double *t = th64 + (size_t)b * kTh;
    t[0] = wb;
    for (int j = 0; j < 4; ++j) t[1 + j] = m[j];
    for (int j = 0; j < 10; ++j) t[5 + j] = C[j];
    t[15] = wb;
    shift[b] = make_float4((float)m[0], (float)m[1], (float)m[2], (float)m[3]);
  }
  double s = 0.0, mx = cb;
  block_sum_max<kUpdThreads>(s, mx, scratch);
  if (act) q[4] = isfinite(cb) ? (float)((cb - mx) * kLog2e) : -INFINITY;
  if (b == 0) {
    const double Cmax = isfinite(mx) ? (mx - 2.0 * kLn2Pi) * kLog2e : 0.0;
    *reinterpret_cast<double *>(cpar + (size_t)K * kPar) = Cmax;
  }
}

// ------------------------------------------------- conditional intensity
// Per component (from the 4D Cholesky factor L of Sigma, whose leading 3 x 3
// block is the factor of Sigma^xx): with z = L_xx^-1 (x - mu^x),
//   ln(pi_b N(x | mu^x, Sigma^xx)) = ln pi_b - 3/2 ln 2pi + sum ln (L_xx^-1)_jj - |z|^2 / 2,
//   m_b(x) = mu^i + L_ix z  (= mu^i + Sigma^ix (Sigma^xx)^-1 (x - mu^x)),
//   v_b = L_ii^2           (= Sigma^ii - Sigma^ix (Sigma^xx)^-1 Sigma^xi).
// Block layout (16 floats): mu^x (3), c' = log2(e) (c_b - C), P' (6, scaled
// by s = sqrt(log2(e)/2)), mu^i, L_ix / s (3), v_b, pad.
constexpr int kCond = 16;

__global__ __launch_bounds__(kUpdThreads) void cond_prep_kernel(
    const float *__restrict__ w, const float *__restrict__ mu,
    const float *__restrict__ cov, int K, float *__restrict__ cb_out,
    uint32_t *status) {
  __shared__ double scratch[2 * kUpdThreads / 64];
  const int b = threadIdx.x;
  const bool act = b < K;
  double cb = -INFINITY;
  float *q = cb_out + (size_t)b * kCond;
  if (act) {
    double C[10], L[10], P[10];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c <= r; ++c) C[tri(r, c)] = cov[16 * b + 4 * r + c];
    const double wb = w[b];
    if (!(wb > 0.0) || !isfinite(wb)) set_status(status, kStBadArg);
    if (chol_inv4(C, L, P)) {
      const double s = sqrt(0.5 * kLog2e);
      for (int j = 0; j < 3; ++j) q[j] = mu[4 * b + j];
      // the leading 3 x 3 block of P = L^-1 is L_xx^-1
      q[4] = (float)(s * P[tri(0, 0)]);
      q[5] = (float)(s * P[tri(1, 0)]);
      q[6] = (float)(s * P[tri(1, 1)]);
      q[7] = (float)(s * P[tri(2, 0)]);
      q[8] = (float)(s * P[tri(2, 1)]);
      q[9] = (float)(s * P[tri(2, 2)]);
      q[10] = mu[4 * b + 3];
      for (int j = 0; j < 3; ++j) q[11 + j] = (float)(L[tri(3, j)] / s);
      q[14] = (float)(L[tri(3, 3)] * L[tri(3, 3)]);
      q[15] = 0.0f;
      cb = log(wb * P[tri(0, 0)] * P[tri(1, 1)] * P[tri(2, 2)]);
    } else {
      // a component that is not SPD takes no part (weight 2^-inf = 0)
      for (int j = 0; j < kCond; ++j) q[j] = 0.0f;
      set_status(status, kStNotSpd);
    }
  }
  double sdum = 0.0, mx = cb;
  block_sum_max<kUpdThreads>(sdum, mx, scratch);
  if (act) q[3] = isfinite(cb) ? (float)((cb - mx) * kLog2e) : -INFINITY;
}

__device__ __forceinline__ float cond_logterm(const float *__restrict__ q, float x, float y,
                                              float z, float &m) {
  const float d0 = x - q[0], d1 = y - q[1], d2 = z - q[2];
  const float z0 = q[4] * d0;
  const float z1 = fmaf(q[5], d0, q[6] * d1);
  const float z2 = fmaf(q[7], d0, fmaf(q[8], d1, q[9] * d2));
  m = fmaf(q[11], z0, fmaf(q[12], z1, fmaf(q[13], z2, q[10])));
  float l = fmaf(-z0, z0, q[3]);
  l = fmaf(-z1, z1, l);
  return fmaf(-z2, z2, l);
}

// One thread per location: beta_b = softmax of the marginal log terms,
// E = sum beta m_b, V = sum beta (v_b + (m_b - E)^2), with FP64 sums.
__global__ __launch_bounds__(256) void cond4_kernel(const float *__restrict__ locs, int64_t M,
                                                    const float *__restrict__ cb, int K,
                                                    float *__restrict__ Eout,
                                                    float *__restrict__ Vout,
                                                    uint32_t *status) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const float x = locs[3 * i], y = locs[3 * i + 1], z = locs[3 * i + 2];
  if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
    set_status(status, kStNonFinite);
    Eout[i] = NAN;
    Vout[i] = NAN;
    return;
  }
  float shift = 0.0f;
  double s = 0.0, s1 = 0.0, s2 = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    s = 0.0; s1 = 0.0; s2 = 0.0;
    for (int b = 0; b < K; ++b) {
      const float *q = cb + (size_t)b * kCond;
      float m;
      const float l = cond_logterm(q, x, y, z, m);
      const double e = (double)__builtin_amdgcn_exp2f(l - shift);
      s += e;
      s1 += e * (double)m;
      s2 = fma(e, (double)q[14] + (double)m * (double)m, s2);
    }
    if (s >= 0x1p-100) break;
    // far from every component: redo with this location's own maximum
    float mx = -INFINITY;
    for (int b = 0; b < K; ++b) {
      float m;
      mx = fmaxf(mx, cond_logterm(cb + (size_t)b * kCond, x, y, z, m));
    }
    shift = mx;
  }
  const double E = s1 / s;
  // variance of the mixture, centred in FP64 (the raw second moment and
  // E^2 are both O(E^2))
  double V = s2 / s - E * E;
  if (V < 0.0) V = 0.0;
  Eout[i] = (float)E;
  Vout[i] = (float)V;
}

// ----------------------------------------------------------- joint sampling
// run[b] = w_0 + ... + w_b in double, component order (one thread), and the
// FP64 Cholesky factors (lower, 10 values) per component.
__global__ __launch_bounds__(256) void sample_prep_kernel(const float *__restrict__ w,
                                                          const float *__restrict__ cov, int K,
                                                          double *__restrict__ run,
                                                          double *__restrict__ Lf,
                                                          int *__restrict__ last,
                                                          uint32_t *status) {
  for (int b = threadIdx.x; b < K; b += blockDim.x) {
    double C[10], L[10], P[10];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c <= r; ++c) C[tri(r, c)] = cov[16 * b + 4 * r + c];
    if (!chol_inv4(C, L, P)) {
      set_status(status, kStNotSpd);
      for (int j = 0; j < 10; ++j) L[j] = NAN;
    }
    for (int j = 0; j < 10; ++j) Lf[10 * b + j] = L[j];
    if (!(w[b] >= 0.0f) || !isfinite(w[b])) set_status(status, kStBadArg);
  }
  if (threadIdx.x == 0) {
    double acc = 0.0;
    int lp = -1;
    for (int b = 0; b < K; ++b) {
      acc += (double)w[b];
      run[b] = acc;
      if (w[b] > 0.0f) lp = b;
    }
    if (lp < 0) set_status(status, kStBadArg);
    *last = lp < 0 ? 0 : lp;
  }
}

// One thread per sample: the first component whose running weight sum
// exceeds u W (binary search over run), then mu_b + L_b z in FP64.
__global__ __launch_bounds__(256) void sample4_kernel(
    const double *__restrict__ run, const double *__restrict__ Lf,
    const int *__restrict__ last, const float *__restrict__ mu, int K, int64_t M,
    const double *__restrict__ u, const float *__restrict__ zin, float *__restrict__ out,
    int32_t *__restrict__ comp, uint32_t *status) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const double ui = u[i];
  if (!(ui >= 0.0 && ui < 1.0)) set_status(status, kStBadArg);
  const double t = ui * run[K - 1];
  int lo = 0, hi = K;  // first index in [lo, hi) with run > t
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (run[mid] > t) hi = mid;
    else lo = mid + 1;
  }
  const int b = lo < K ? lo : *last;
  const double *L = Lf + 10 * b;
  double zz[4];
  for (int j = 0; j < 4; ++j) zz[j] = (double)zin[4 * i + j];
  for (int r = 0; r < 4; ++r) {
    double v = (double)mu[4 * b + r];
    for (int c = 0; c <= r; ++c) v = fma(L[tri(r, c)], zz[c], v);
    out[4 * i + r] = (float)v;
  }
  if (comp) comp[i] = b;
}

// ------------------------------------------------------- culled passes
// A soft pass that skips the (tile, component) pairs whose FP32 weight is
// exactly zero for every point of the tile, as the 3D culled kernel does.
// The first three rows of the lower-triangular P' involve x, y, z only, so
// |P'(x - mu)|^2 >= |P'_3 (x_3 - mu_3)|^2 with P'_3 its leading 3 x 3 block
// (the xyz marginal's factor), and for every point whose xyz part lies in a
// sphere (c, r): |P'_3 (x_3 - mu_3)| >= |P'_3 (c - mu_3)| - |P'_3|_F r.
// Where c'_b - max(0, that)^2 is below kCull4Log2 (two units under the
// smallest FP32 subnormal exponent) every e_pb of the tile rounds to zero;
// skipping the pair changes nothing beyond the order of FP32 additions.
// Tiles are 64 points of a cloud in Morton order of its xyz part.
constexpr float kCull4Log2 = -152.0f;
constexpr int kOrd = 256;            // threads of the ordering kernels
constexpr int kBox4Blocks = 256;
constexpr int kCull4Cap = 128;       // E rows kept per tile at most
constexpr int kCull4Waves = 8;       // waves per block (16 measured no faster at K = 505)

__device__ inline void box4_reduce(float *lo, float *hi, float *sh /* 4 x 6 */) {
  for (int off = 32; off > 0; off >>= 1)
    for (int j = 0; j < 3; ++j) {
      lo[j] = fminf(lo[j], __shfl_xor(lo[j], off, 64));
      hi[j] = fmaxf(hi[j], __shfl_xor(hi[j], off, 64));
    }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int j = 0; j < 3; ++j) {
      sh[w * 6 + j] = lo[j];
      sh[w * 6 + 3 + j] = hi[j];
    }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int v = 1; v < kOrd / 64; ++v)
      for (int j = 0; j < 3; ++j) {
        lo[j] = fminf(lo[j], sh[v * 6 + j]);
        hi[j] = fmaxf(hi[j], sh[v * 6 + 3 + j]);
      }
}

// Partial xyz boxes of the n points: part6[block] = (lo, hi).
__global__ __launch_bounds__(kOrd) void bbox4_kernel(const float4 *__restrict__ pts, int64_t n,
                                                     float *__restrict__ part6) {
  __shared__ float sh[kOrd / 64 * 6];
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * kOrd + threadIdx.x; i < n; i += (int64_t)gridDim.x * kOrd) {
    const float4 x = pts[i];
    lo[0] = fminf(lo[0], x.x); lo[1] = fminf(lo[1], x.y); lo[2] = fminf(lo[2], x.z);
    hi[0] = fmaxf(hi[0], x.x); hi[1] = fmaxf(hi[1], x.y); hi[2] = fmaxf(hi[2], x.z);
  }
  box4_reduce(lo, hi, sh);
  if (threadIdx.x == 0)
    for (int j = 0; j < 3; ++j) {
      part6[blockIdx.x * 6 + j] = lo[j];
      part6[blockIdx.x * 6 + 3 + j] = hi[j];
    }
}

__device__ inline unsigned spread3_4(unsigned v) {
  v &= 0xFFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// keys[i] = Morton code of the xyz part of point i in a cubic 256^3 grid
// over the box (0xFFFFFF past the last point, so padding sorts last);
// vals[i] = i.
__global__ __launch_bounds__(kOrd) void morton4_kernel(
    const float4 *__restrict__ pts, int64_t n, int64_t npad, const float *__restrict__ part6,
    int nbox, unsigned *__restrict__ keys, unsigned *__restrict__ vals) {
  __shared__ float sh[kOrd / 64 * 6];
  __shared__ float box[4];
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nbox; b += kOrd)
    for (int j = 0; j < 3; ++j) {
      lo[j] = fminf(lo[j], part6[b * 6 + j]);
      hi[j] = fmaxf(hi[j], part6[b * 6 + 3 + j]);
    }
  box4_reduce(lo, hi, sh);
  if (threadIdx.x == 0) {
    const float ext = fmaxf(fmaxf(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
    box[0] = lo[0];
    box[1] = lo[1];
    box[2] = lo[2];
    box[3] = (ext > 0.0f && ext < INFINITY) ? 255.99f / ext : 0.0f;
  }
  __syncthreads();
  const float l0 = box[0], l1 = box[1], l2 = box[2], sc = box[3];
  for (int64_t i = (int64_t)blockIdx.x * kOrd + threadIdx.x; i < npad;
       i += (int64_t)gridDim.x * kOrd) {
    unsigned key = 0xFFFFFFu;
    if (i < n) {
      const float4 x = pts[i];
      const unsigned q0 = (unsigned)fminf(fmaxf((x.x - l0) * sc, 0.0f), 255.0f);
      const unsigned q1 = (unsigned)fminf(fmaxf((x.y - l1) * sc, 0.0f), 255.0f);
      const unsigned q2 = (unsigned)fminf(fmaxf((x.z - l2) * sc, 0.0f), 255.0f);
      key = spread3_4(q0) | (spread3_4(q1) << 1) | (spread3_4(q2) << 2);
    }
    keys[i] = key;
    vals[i] = (unsigned)i;
  }
}

// out[i] = in[perm[i]] (zero past the n points), labels likewise.
__global__ __launch_bounds__(kOrd) void gather4_kernel(
    const float4 *__restrict__ in, const int32_t *__restrict__ lab_in,
    const unsigned *__restrict__ perm, int64_t n, int64_t npad, float4 *__restrict__ out,
    int32_t *__restrict__ lab_out) {
  const int64_t i = (int64_t)blockIdx.x * kOrd + threadIdx.x;
  if (i >= npad) return;
  const int64_t j = perm[i];
  out[i] = j < n ? in[j] : make_float4(0.f, 0.f, 0.f, 0.f);
  if (lab_out) lab_out[i] = (lab_in && j < n) ? lab_in[j] : 0;
}

// Bounding sphere (xyz centre, radius) of every 64-point tile of the
// ordered points, radius -1 when the tile holds no finite point.  One wave
// per tile.
__global__ __launch_bounds__(kOrd) void tile_sphere4_kernel(const float4 *__restrict__ pts,
                                                            int64_t n, int ntiles,
                                                            float4 *__restrict__ sph) {
  const int t = blockIdx.x * (kOrd / 64) + (threadIdx.x >> 6);
  if (t >= ntiles) return;   // uniform per wave
  const int64_t i = (int64_t)t * kT + (threadIdx.x & 63);
  float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
  bool ok = false;
  if (i < n) {
    x = pts[i];
    ok = isfinite(x.x) && isfinite(x.y) && isfinite(x.z) && isfinite(x.w);
  }
  float lo0 = ok ? x.x : INFINITY, lo1 = ok ? x.y : INFINITY, lo2 = ok ? x.z : INFINITY;
  float hi0 = ok ? x.x : -INFINITY, hi1 = ok ? x.y : -INFINITY, hi2 = ok ? x.z : -INFINITY;
  for (int off = 32; off > 0; off >>= 1) {
    lo0 = fminf(lo0, __shfl_xor(lo0, off, 64));
    lo1 = fminf(lo1, __shfl_xor(lo1, off, 64));
    lo2 = fminf(lo2, __shfl_xor(lo2, off, 64));
    hi0 = fmaxf(hi0, __shfl_xor(hi0, off, 64));
    hi1 = fmaxf(hi1, __shfl_xor(hi1, off, 64));
    hi2 = fmaxf(hi2, __shfl_xor(hi2, off, 64));
  }
  if ((threadIdx.x & 63) != 0) return;
  if (!(lo0 <= hi0)) {
    sph[t] = make_float4(0.f, 0.f, 0.f, -1.0f);
    return;
  }
  const float c0 = 0.5f * (lo0 + hi0), c1 = 0.5f * (lo1 + hi1), c2 = 0.5f * (lo2 + hi2);
  const float e0 = hi0 - lo0, e1 = hi1 - lo1, e2 = hi2 - lo2;
  // half diagonal, widened for the rounding of the centre and the norm
  const float scale = fmaxf(fmaxf(fabsf(c0), fabsf(c1)), fabsf(c2)) + 1.0f;
  const float r = 0.5f * sqrtf(e0 * e0 + e1 * e1 + e2 * e2) * (1.0f + 1e-5f) + 1e-5f * scale;
  sph[t] = make_float4(c0, c1, c2, r);
}

struct Cull4Args {
  int64_t n;
  int ntiles, K, mode, ncols, scap;
  int cmaj;   // partial row component-major (b kNStat + j), for the fused update
};

// LDS of the culled kernel: FP64 sums (K x kNStat) | E rows (scap x kTS) |
// Xs (kT float4) | Rs (kT) | partial normalisers (8 x kT) | far-point
// (max, sum) (kT float2) | per-wave chunk lists (8 x 64 uint16) | slot ->
// component (kMaxK uint16) | chunk counts (8) | far-point mask | wL (8).
struct Cull4Lds {
  size_t acc, E, Xs, Rs, reds, fbv, lst, comp, cnt, fbm, wL, total;
};
__host__ __device__ inline Cull4Lds cull4_lds(int K, int scap, int nw) {
  Cull4Lds L{};
  size_t o = 0;
  auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
  L.acc = o; o = al(o + (size_t)K * kNStat * sizeof(double));
  L.E = o; o = al(o + (size_t)scap * kTS * sizeof(float));
  L.Xs = o; o = al(o + kT * sizeof(float4));
  L.Rs = o; o = al(o + kT * sizeof(float));
  L.reds = o; o = al(o + (size_t)nw * kT * sizeof(float));
  L.fbv = o; o = al(o + kT * sizeof(float2));
  L.lst = o; o = al(o + (size_t)nw * 64 * sizeof(uint16_t));
  L.comp = o; o = al(o + kMaxK * sizeof(uint16_t));
  L.cnt = o; o = al(o + (size_t)nw * sizeof(int));
  L.fbm = o; o = al(o + sizeof(unsigned long long));
  L.wL = o; o = al(o + (size_t)nw * sizeof(double));
  L.total = o;
  return L;
}

// One culled soft pass (E+M statistics, or L only), grid-strided over the
// 64-point tiles, NW waves per block.  Per tile, four barriers:
//  cull    wave g < ceil(K / 64) tests components 64 g .. 64 g + 63
//          (parameters held in registers for the whole launch) against the
//          tile's sphere and writes its active components, in order, to its
//          own chunk list |
//  E-phase the active components taken in chunk order form slots 0 ..
//          nact - 1; wave g takes slots g, g + NW, ... for the tile's 64
//          points and stores e_pb in LDS row `slot` (rows for scap slots;
//          later rows are recomputed in the M-phase chunk by chunk) |
//  normaliser  wave 0, one lane per point: s_p, 1 / s_p and L; a point
//          with s_p below 2^-100 is left out and added after the M-phase
//          with its own maximum over all K components, as the dense kernel
//          does (one more round over every component, 1 / s_p of those
//          points only) |
//  M-phase lanes = (slot, subset of 8 points): FP32 statistics, summed over
//          the 8 subsets by DPP in a fixed order, added to the FP64 sums.
template <int NW>
__global__ __launch_bounds__(NW * 64) void em4_cull_kernel(
    const float4 *__restrict__ pts, const float4 *__restrict__ sph,
    const float *__restrict__ cpar, const float4 *__restrict__ shift,
    double *__restrict__ part, Cull4Args a) {
  constexpr int G = NW, BLOCK = NW * 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int K = a.K, mode = a.mode, scap = a.scap;
  const Cull4Lds LL = cull4_lds(K, scap, NW);
  double *acc = reinterpret_cast<double *>(smem + LL.acc);
  float *E = reinterpret_cast<float *>(smem + LL.E);
  float4 *Xs = reinterpret_cast<float4 *>(smem + LL.Xs);
  float *Rs = reinterpret_cast<float *>(smem + LL.Rs);
  float *reds = reinterpret_cast<float *>(smem + LL.reds);
  float2 *fbv = reinterpret_cast<float2 *>(smem + LL.fbv);
  uint16_t *lst = reinterpret_cast<uint16_t *>(smem + LL.lst);
  uint16_t *comp = reinterpret_cast<uint16_t *>(smem + LL.comp);
  int *cnt = reinterpret_cast<int *>(smem + LL.cnt);
  unsigned long long *fbm = reinterpret_cast<unsigned long long *>(smem + LL.fbm);
  double *wL = reinterpret_cast<double *>(smem + LL.wL);

  const int tid = threadIdx.x, lane = tid & 63;
  const int g = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double Cb = *reinterpret_cast<const double *>(cpar + (size_t)K * kPar);
  // cull parameters of component 64 g + lane: mu_xyz, c', P'_3, |P'_3|_F
  const int cb = g * 64 + lane;
  float m0 = 0.f, m1 = 0.f, m2 = 0.f, cc = -INFINITY;
  float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f, p4 = 0.f, p5 = 0.f, fro = 0.f;
  if (cb < K) {
    const float *q = cpar + (size_t)cb * kPar;
    m0 = q[0]; m1 = q[1]; m2 = q[2]; cc = q[4];
    p0 = q[5]; p1 = q[6]; p2 = q[7]; p3 = q[8]; p4 = q[9]; p5 = q[10];
    fro = sqrtf(p0 * p0 + p1 * p1 + p2 * p2 + p3 * p3 + p4 * p4 + p5 * p5);
  }
  for (int i = tid; i < K * kNStat; i += BLOCK) acc[i] = 0.0;
  double Lacc = 0.0;
  __syncthreads();

  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int64_t idx = (int64_t)tile * kT + lane;
    float4 x = idx < a.n ? pts[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
    const bool valid = idx < a.n && isfinite(x.x) && isfinite(x.y) && isfinite(x.z) &&
                       isfinite(x.w);
    if (!valid) x = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 sp = sph[tile];
    // ---- cull: this wave's chunk of components
    bool keep = false;
    if (g * 64 < K && sp.w >= 0.0f) {
      const float d0 = sp.x - m0, d1 = sp.y - m1, d2 = sp.z - m2;
      const float z0 = p0 * d0;
      const float z1 = fmaf(p1, d0, p2 * d1);
      const float z2 = fmaf(p3, d0, fmaf(p4, d1, p5 * d2));
      const float dist = sqrtf(fmaf(z0, z0, fmaf(z1, z1, z2 * z2)));
      const float bnd = fmaxf(dist - fro * sp.w, 0.0f);
      keep = fmaf(-bnd, bnd, cc) >= kCull4Log2;
    }
    const uint64_t km = __ballot(keep);
    if (keep) {
      const unsigned below = __builtin_amdgcn_mbcnt_hi(
          (unsigned)(km >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)km, 0u));
      lst[g * 64 + (int)below] = (uint16_t)cb;
    }
    if (lane == 0) cnt[g] = __popcll(km);
    __syncthreads();                                                  // 1

    // ---- slots: the chunk lists one after another
    int pre[G + 1];
    pre[0] = 0;
#pragma unroll
    for (int j = 0; j < G; ++j) pre[j + 1] = pre[j] + __builtin_amdgcn_readfirstlane(cnt[j]);
    const int nact = pre[G];
    float s = 0.0f;
    for (int r = g; r < nact; r += G) {
      int base = 0, off = 0;
#pragma unroll
      for (int j = 1; j < G; ++j)
        if (r >= pre[j]) {
          base = j * 64;
          off = pre[j];
        }
      const int b = __builtin_amdgcn_readfirstlane((int)lst[base + r - off]);
      const float e = __builtin_amdgcn_exp2f(logterm4(cpar + (size_t)b * kPar, x));
      s += e;
      if (r < scap) E[r * kTS + lane] = e;
      if (lane == 0) comp[r] = (uint16_t)b;
    }
    reds[g * kT + lane] = s;
    __syncthreads();                                                  // 2

    // ---- normaliser (wave 0)
    if (g == 0) {
      float st = reds[lane];
#pragma unroll
      for (int j = 1; j < G; ++j) st += reds[j * kT + lane];
      const bool fb = valid && !(st >= 0x1p-100f);
      float mref = 0.0f;
      if (fb) {
        float mx = -INFINITY;
        for (int bb = 0; bb < K; ++bb) mx = fmaxf(mx, logterm4(cpar + (size_t)bb * kPar, x));
        st = 0.0f;
        for (int bb = 0; bb < K; ++bb)
          st += __builtin_amdgcn_exp2f(logterm4(cpar + (size_t)bb * kPar, x) - mx);
        mref = mx;
        fbv[lane] = make_float2(mx, st);
      }
      Xs[lane] = x;
      Rs[lane] = (valid && !fb) ? __builtin_amdgcn_rcpf(st) : 0.0f;
      const uint64_t fm = __ballot(fb);
      if (lane == 0) *fbm = fm;
      if (valid) Lacc += (Cb + (double)mref + (double)__builtin_amdgcn_logf(st)) * kLn2;
    }
    __syncthreads();                                                  // 3

    // ---- M-phase
    const uint64_t fmask = *fbm;
    // E rows of slots [c0, c0 + nloc), the normaliser being known; far:
    // slot = component, e = 2^(l - m_p) for the far points (max m_p)
    auto rows = [&](int c0, int nloc, bool far) {
      for (int u = tid; u < nloc * kT; u += BLOCK) {
        const int sl = u >> 6, p2 = u & 63;
        const int b = far ? c0 + sl : comp[c0 + sl];
        const float off = (far && ((fmask >> p2) & 1ull)) ? fbv[p2].x : 0.0f;
        E[sl * kTS + p2] =
            __builtin_amdgcn_exp2f(logterm4(cpar + (size_t)b * kPar, Xs[p2]) - off);
      }
    };
    // statistics of slots [c0, c0 + nloc) from rows 0 .. nloc - 1
    auto stats = [&](int c0, int nloc, bool far) {
      const int q = tid & 7;
      for (int s0 = 0; s0 < nloc; s0 += BLOCK / 8) {
        const int sl = s0 + (tid >> 3);
        if (sl < nloc) {
          const int b = far ? c0 + sl : comp[c0 + sl];
          const float4 sh = shift[b];
          const float *Eb = E + sl * kTS + q * 8;
          const float4 *Xb = Xs + q * 8;
          const float *Rb = Rs + q * 8;
          float v[kNStat];
#pragma unroll
          for (int j = 0; j < kNStat; ++j) v[j] = 0.0f;
#pragma unroll 2
          for (int j = 0; j < 8; ++j) {
            const float4 xr = Xb[j];
            const float gm = Eb[j] * Rb[j];
            const float d[4] = {xr.x - sh.x, xr.y - sh.y, xr.z - sh.z, xr.w - sh.w};
            v[0] += gm;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float wr = gm * d[r];
              v[1 + r] += wr;
#pragma unroll
              for (int c = 0; c <= r; ++c) v[5 + tri(r, c)] = fmaf(wr, d[c], v[5 + tri(r, c)]);
            }
          }
          // sum over the slot's 8 lanes as a reduce-scatter: each exchange
          // (lane 7 - l of the half row, then l ^ 2, then l ^ 1) keeps the
          // half of the statistics that this side owns; lane q ends with
          // statistics 2q and 2q + 1 (statistic 15 is padding)
          const bool b4 = (q & 4) != 0, b2 = (q & 2) != 0, b1 = (q & 1) != 0;
          float k8[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const float hi = (j + 8 < kNStat) ? v[j + 8] : 0.0f;
            const float keep = b4 ? hi : v[j], send = b4 ? v[j] : hi;
            k8[j] = keep + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(send), 0x141,
                                                                   0xF, 0xF, true));
          }
          float k4[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float keep = b2 ? k8[j + 4] : k8[j], send = b2 ? k8[j] : k8[j + 4];
            k4[j] = keep + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(send), 0x4E,
                                                                   0xF, 0xF, true));
          }
          float k2[2];
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const float keep = b1 ? k4[j + 2] : k4[j], send = b1 ? k4[j] : k4[j + 2];
            k2[j] = keep + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(send), 0xB1,
                                                                   0xF, 0xF, true));
          }
          double *ab = acc + (size_t)b * kNStat;
          ab[2 * q] += (double)k2[0];
          if (2 * q + 1 < kNStat) ab[2 * q + 1] += (double)k2[1];
        }
      }
    };
    if (mode != kSoftLogLik) {
      // rounds of scap slots: the active components, then (rare) every
      // component once more for the far points, 1 / s_p of those only
      const int nnorm = (nact + scap - 1) / scap;
      const int nrd = nnorm + (fmask != 0ull ? (K + scap - 1) / scap : 0);
      for (int rd = 0; rd < nrd; ++rd) {
        const bool far = rd >= nnorm;
        const int c0 = (far ? rd - nnorm : rd) * scap;
        const int nloc = min(scap, (far ? K : nact) - c0);
        if (rd > 0 || far) {
          if (rd > 0) __syncthreads();   // the previous rows and Rs consumed
          if (far && rd == nnorm && g == 0)
            Rs[lane] = ((fmask >> lane) & 1ull) ? __builtin_amdgcn_rcpf(fbv[lane].y) : 0.0f;
          rows(c0, nloc, far);
          __syncthreads();
        }
        stats(c0, nloc, far);
      }
    }
    __syncthreads();                                                  // 4
  }

  double *row = part + (size_t)blockIdx.x * a.ncols;
  if (mode != kSoftLogLik) {
    if (a.cmaj) {
      for (int i = tid; i < K * kNStat; i += BLOCK) row[i] = acc[i];
    } else {
      for (int i = tid; i < K * kNStat; i += BLOCK) {
        const int j = i / K, b = i - j * K;
        row[i] = acc[(size_t)b * kNStat + j];
      }
    }
  }
  double v = Lacc;
  v = wave_sum_f64(v);
  if (lane == 0) wL[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int j = 0; j < G; ++j) sum += wL[j];
    row[kNStat * K] = sum;
  }
}

}  // namespace gmm4_dev
