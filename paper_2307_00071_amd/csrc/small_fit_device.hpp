// Small fits in one launch: every soft EM iteration (eq. 2 E-step, the
// M-step of Sec. V: weights, means, covariances with lambda I, Cholesky)
// of a fit with K <= 16 components and at most 256 tiles of 256 points.
//
// For such fits a launch pair per iteration (tile pass, reduction + M-step)
// costs more than its arithmetic.  Here one block owns one 256-point tile
// for the whole fit and keeps its point in a register.  Per iteration:
//  E-phase  thread p: l'_pb for every component from the parameters in LDS,
//           e_pb = 2^l'_pb into the LDS row of b, s_p, lse_p (a point whose
//           s_p underflows is redone with its own maximum, as in the tile
//           kernel);
//  M-phase  thread (b, q): the ten shifted sums of component b over point
//           subset q (FP32 over at most 16 points, then FP64), the P
//           subsets added in order, and the block's log-likelihood sum:
//           one FP64 partial row of 10 K + 1 values;
//  barrier  wave 0 stores the row (rows alternate between two buffers by
//           iteration parity), releases it at device scope and takes a
//           ticket; the block waits until every block's ticket for this
//           iteration is in (bounded: after kSmallSpinLimit polls, or when
//           another block gave up, the block sets the device-error bit and
//           returns, so every wave exits);
//  update   every block adds all rows in the same fixed order and runs the
//           same FP64 M-step into its own LDS parameters, so no block reads
//           parameters another block wrote during the launch; block 0 also
//           writes the log-likelihood of the iteration, the FP64 state and,
//           after the last iteration, the E-step block for the next launch;
//  stop     with a tolerance, every block makes the same decision from the
//           same L.
// All blocks must be resident at once: the host launches at most one
// block per compute unit.

#pragma once

#include "em_device.hpp"

namespace gmm_dev {

constexpr int kSmallThreads = 256;     // block = tile = 256 points
constexpr int kSmallMaxK = 16;
constexpr int kSmallMaxTiles = 256;    // blocks (one tile each)
constexpr int kSmallTS = kSmallThreads + 1;   // odd LDS row stride
constexpr unsigned kSmallSpinLimit = 1u << 22;
constexpr uint32_t kStDevice = 1u << GMM_ERR_DEVICE;

struct SmallArgs {
  int K, P, trip, iters, ncols;
  double reg;
  // > 0: stopping rule; after the M-step of the first iteration t >= 1 with
  // |L_t - L_(t-1)| <= tol_abs the fit keeps theta_(t+1), and the L of the
  // skipped iterations is NaN
  double tol_abs;
  // tests of the give-up path: at this iteration block 0 raises the flag
  // instead of taking its ticket (-1: never)
  int give_up_at;
};

__global__ __launch_bounds__(kSmallThreads) void em_small_fit_kernel(
    const float4 *__restrict__ pts, const float *__restrict__ cpar_in,
    const float4 *__restrict__ shift_in, float *__restrict__ cpar_out,
    float4 *__restrict__ shift_out, double *__restrict__ th64,
    double *__restrict__ part, unsigned *__restrict__ bar,
    double *__restrict__ loglik, uint32_t *__restrict__ status, SmallArgs a) {
  constexpr int NT = kSmallThreads, TS = kSmallTS;
  static_assert(NT == 256, "the log-likelihood sum adds four wave sums");
  constexpr int NPAR = (kSmallMaxK + 1) * kParStride;
  __shared__ __align__(16) float cp[2][NPAR];
  __shared__ float4 sh[2][kSmallMaxK];
  __shared__ float E[kSmallMaxK * TS];
  __shared__ float4 Xs[NT];
  __shared__ double D[NT * kNStat];
  __shared__ double row[kNStat * kSmallMaxK + 1];
  __shared__ double tot[kNStat * kSmallMaxK + 1];
  __shared__ double thl[kSmallMaxK * kTh64Stride];
  __shared__ double scr[2 * NT / 64 + 2];
  __shared__ int abort_flag;

  const int tid = threadIdx.x, lane = tid & 63;
  const int K = a.K, P = a.P, trip = a.trip, ncols = a.ncols;
  const int grid = gridDim.x, blk = blockIdx.x;
  const int nf = (K + 1) * kParStride;
  for (int i = tid; i < nf; i += NT) cp[0][i] = cpar_in[i];
  if (tid < K) sh[0][tid] = shift_in[tid];
  if (tid == 0) abort_flag = 0;
  const float4 x = pts[(size_t)blk * NT + tid];
  const bool valid = __float_as_int(x.w) >= 0;
  const bool mact = tid < K * P;
  const int mb = mact ? tid % K : 0, mq = mact ? tid / K : 0;
  // a statistic column c = s K + b of the row; the P subset sums of
  // component b, statistic s are at D[(q K + b) kNStat + s]
  const int cs = tid / K, cb = tid - (tid / K) * K;
  double *th_mine = blk == 0 ? th64 : thl;
  int cur = 0;
  double Lprev = 0.0;
  __syncthreads();

  for (int t = 0; t < a.iters; ++t) {
    const float *cq = cp[cur];
    // ---- E-phase
    const double Cb = *reinterpret_cast<const double *>(cq + (size_t)K * kParStride);
    float s = 0.0f;
#pragma unroll 4
    for (int b = 0; b < K; ++b) {
      const float e = __builtin_amdgcn_exp2f(
          comp_logterm(cq + b * kParStride, x.x, x.y, x.z));
      E[b * TS + tid] = e;
      s += e;
    }
    float mref = 0.0f;
    if (valid && !(s >= 0x1p-100f)) {
      float m = -INFINITY;
      for (int b = 0; b < K; ++b)
        m = fmaxf(m, comp_logterm(cq + b * kParStride, x.x, x.y, x.z));
      s = 0.0f;
      for (int b = 0; b < K; ++b) {
        const float e = __builtin_amdgcn_exp2f(
            comp_logterm(cq + b * kParStride, x.x, x.y, x.z) - m);
        E[b * TS + tid] = e;
        s += e;
      }
      mref = m;
    }
    Xs[tid] = make_float4(x.x, x.y, x.z, valid ? __builtin_amdgcn_rcpf(s) : 0.0f);
    const double lse =
        valid ? (Cb + (double)mref + (double)__builtin_amdgcn_logf(s)) * kLn2 : 0.0;
    __syncthreads();
    // ---- M-phase: subset q of component b
    if (mact) {
      const float4 m = sh[cur][mb];
      const float *Eb = E + mb * TS + mq * trip;
      const float4 *Xb = Xs + mq * trip;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f, a5 = 0.f,
            a6 = 0.f, a7 = 0.f, a8 = 0.f, a9 = 0.f;
#pragma unroll 4
      for (int j = 0; j < trip; ++j) {
        const float4 xr = Xb[j];
        const float gm = Eb[j] * xr.w;
        const float d0 = xr.x - m.x, d1 = xr.y - m.y, d2 = xr.z - m.z;
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
      double *d = D + (size_t)(mq * K + mb) * kNStat;
      d[0] = a0; d[1] = a1; d[2] = a2; d[3] = a3; d[4] = a4;
      d[5] = a5; d[6] = a6; d[7] = a7; d[8] = a8; d[9] = a9;
    }
    // the block's log-likelihood: wave sums (DPP rows, then rows in order),
    // then the waves in order
    const double wl = wave_sum_f64(lse);
    if (lane == 0) scr[tid >> 6] = wl;
    __syncthreads();
    if (tid < kNStat * K) {
      double acc = 0.0;
#pragma unroll 8
      for (int q = 0; q < P; ++q) acc += D[(size_t)(q * K + cb) * kNStat + cs];
      row[tid] = acc;
    }
    if (tid == 0) row[kNStat * K] = (scr[0] + scr[1]) + (scr[2] + scr[3]);
    __syncthreads();
    // ---- grid barrier (wave 0)
    double *rows = part + (size_t)(t & 1) * grid * ncols;
    if (tid < 64) {
      for (int c = lane; c < ncols; c += 64) rows[(size_t)blk * ncols + c] = row[c];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (lane == 0 && blk == 0 && t == a.give_up_at) {
        __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        abort_flag = 1;
      } else if (lane == 0) {
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = (unsigned)(t + 1) * (unsigned)grid;
        unsigned spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
          if (++spins > kSmallSpinLimit ||
              __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            abort_flag = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
    __syncthreads();
    if (abort_flag) {
      if (tid == 0) set_status(status, kStDevice);
      return;
    }
    // (lane 0's acquire, then the workgroup barrier: every wave of the
    // block reads the rows after that)
    // ---- every row: G groups of ncols threads, group g the rows g, g + G,
    // ... in order (all loads of a round in flight), then the G group sums
    // in group order; every block adds identically
    {
      const int G = NT / ncols;
      const int g = tid / ncols, c = tid - g * ncols;
      if (g < G) {
        const double *src = rows + c;
        double acc = 0.0;
        for (int r0 = g; r0 < grid; r0 += 16 * G) {
          double v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u)
            v[u] = (r0 + u * G < grid) ? src[(size_t)(r0 + u * G) * ncols] : 0.0;
#pragma unroll
          for (int u = 0; u < 16; ++u) acc += v[u];
        }
        D[tid] = acc;
      }
      __syncthreads();
      if (tid < ncols) {
        double acc = D[tid];
        for (int h = 1; h < G; ++h) acc += D[h * ncols + tid];
        tot[tid] = acc;
      }
      __syncthreads();
    }
    if (blk == 0 && tid == 0) {
      const double L = tot[kNStat * K];
      if (loglik) loglik[t] = L;
      if (!isfinite(L)) set_status(status, kStNonFinite);
    }
    const int nxt = 1 - cur;
    em_update_block<NT, true>(tot, K, kUpdFull, a.reg, cp[cur], sh[cur], cp[nxt], sh[nxt],
                        th_mine, scr, status);
    cur = nxt;
    // every block holds the same L bits, so all stop at the same iteration
    const double L = tot[kNStat * K];
    const bool stop = a.tol_abs > 0.0 && t >= 1 && fabs(L - Lprev) <= a.tol_abs;
    Lprev = L;
    __syncthreads();
    if (stop) {
      if (blk == 0 && loglik)
        for (int u = t + 1 + tid; u < a.iters; u += NT) loglik[u] = (double)NAN;
      break;
    }
  }
  if (blk == 0) {
    for (int i = tid; i < nf; i += NT) cpar_out[i] = cp[cur][i];
    if (tid < K) shift_out[tid] = sh[cur][tid];
  }
}

}  // namespace gmm_dev
