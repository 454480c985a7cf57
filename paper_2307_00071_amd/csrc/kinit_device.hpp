// kinit_device.hpp - k-means++ seeding on the device (the initialisation
// that precedes EM; the paper starts EM from a randomised k-means step,
// Sec. V).  D^2 seeding after Arthur & Vassilvitskii (2007), one trial per
// centre, hard nearest-seed labels.
//
// With K draws u[j] in [0, 1):
//   centre 0 = floor(u[0] N) (at most N - 1);
//   D2_i = squared distance from x_i to the nearest centre so far;
//   centre j = the first index whose running sum of D2 exceeds u[j] W,
//     W = sum D2 (so index i is drawn with probability D2_i / W); when
//     W = 0 centre j repeats centre j - 1;
//   label_i = the nearest centre, the lowest index on ties.
// The running sums have a fixed order so that the choice is reproducible:
// sequential within chunks of kKppChunk points, chunk totals sequential in
// runs of 16 from offsets formed by a block scan (kpp_select_kernel); the
// pick is the first positive entry above u W, else the last positive entry.
// Squared distances are ((dx^2 + dy^2) + dz^2) in double with every
// operation rounded on its own (no contraction).
//
// Per round j >= 1: kpp_update_kernel (D2 with centre j - 1, chunk totals)
// and kpp_select_kernel (one block: W, the chunk, the point).  The
// update streams 28 B per point per round (the point, D2 read and
// written); the select kernel is a short chain of dependent reads and
// serial sums; neither does enough arithmetic to meet a compute roofline.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmm_dev {

constexpr int kKppChunk = 256;      // points per chunk (running-sum order)
constexpr int kKppSelThreads = 1024;
constexpr int kKppLabelThreads = 256;

__device__ __forceinline__ double kpp_d2(double a0, double a1, double a2, double b0,
                                         double b1, double b2) {
#pragma clang fp contract(off)
  const double d0 = a0 - b0, d1 = a1 - b1, d2 = a2 - b2;
  return (d0 * d0 + d1 * d1) + d2 * d2;
}

// Checks the draws and places centre 0.  One block.
__global__ __launch_bounds__(256) void kpp_first_kernel(const double *__restrict__ u, int K,
                                                        int64_t n, int64_t *__restrict__ cidx,
                                                        uint32_t *status) {
  for (int j = threadIdx.x; j < K; j += 256) {
    const double v = u[j];
    if (!(v >= 0.0 && v < 1.0)) set_status(status, kStBadArg);
  }
  if (threadIdx.x == 0) {
    const double v = u[0];
    int64_t c = (v >= 0.0 && v < 1.0) ? (int64_t)(v * (double)n) : 0;
    cidx[0] = c > n - 1 ? n - 1 : c;
  }
}

// D2 with centre j (the first round sets it) and the chunk totals.  A
// block of kKppUpdThreads threads takes kKppUpdChunks chunks; the D2 values
// go to LDS (one padded row per chunk), then lane c of wave 0 sums chunk c
// sequentially (the chains run side by side in one wave).
constexpr int kKppUpdThreads = 256;
constexpr int kKppUpdChunks = 4;
constexpr int kKppRow = kKppChunk + 1;  // padded LDS row (bank spread)
__global__ __launch_bounds__(kKppUpdThreads) void kpp_update_kernel(
    const float *__restrict__ pts, int64_t n, const int64_t *__restrict__ cidx, int j,
    double *__restrict__ D, double *__restrict__ T, int64_t nch, uint32_t *status) {
  __shared__ double sh[kKppUpdChunks * kKppRow];
  const int64_t c = cidx[j];
  const double c0 = pts[3 * c], c1 = pts[3 * c + 1], c2 = pts[3 * c + 2];
  const int64_t base = (int64_t)blockIdx.x * kKppUpdChunks * kKppChunk;
  constexpr int PER = kKppUpdChunks * kKppChunk / kKppUpdThreads;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int l = q * kKppUpdThreads + threadIdx.x;
    const int64_t i = base + l;
    double v = 0.0;  // past the end: 0, which leaves the running sums as they are
    if (i < n) {
      const float x0 = pts[3 * i], x1 = pts[3 * i + 1], x2 = pts[3 * i + 2];
      const double d = kpp_d2(x0, x1, x2, c0, c1, c2);
      if (j == 0) {
        if (!isfinite(x0) || !isfinite(x1) || !isfinite(x2)) set_status(status, kStNonFinite);
        v = d;
      } else {
        const double o = D[i];
        v = d < o ? d : o;
      }
      D[i] = v;
    }
    sh[(l / kKppChunk) * kKppRow + (l % kKppChunk)] = v;
  }
  __syncthreads();
  const int64_t ch = (int64_t)blockIdx.x * kKppUpdChunks + threadIdx.x;
  if (threadIdx.x < kKppUpdChunks && ch < nch) {
    const double *a = sh + threadIdx.x * kKppRow;
    double s = 0.0;
    for (int k0 = 0; k0 < kKppChunk; k0 += 16) {
      double e[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) e[k] = a[k0 + k];
#pragma unroll
      for (int k = 0; k < 16; ++k) s += e[k];
    }
    T[ch] = s;
  }
}

// ---- centre j >= 1: one block of kKppSelThreads threads.
// The running sums in index order are formed as: chunk totals (sequential
// over 256 points, kpp_update_kernel); kKppSelPer consecutive chunk totals
// per thread of a stage of kKppSelThreads x kKppSelPer chunks, sequential
// from the thread's offset; the thread offsets by a block scan of the
// thread sums (a shuffle scan in each wave, the wave totals in order); the
// stages in order.  Inside the chosen chunk the 256 D2 by the same block
// scan from the chunk's running sum.  The pick is the first positive entry
// whose running sum exceeds t = u_j W (the exact running sum is flat over
// zero entries, so none of them is ever the first above a level); where
// rounding leaves no entry above t, the last positive entry.
constexpr int kKppSelPer = 16;

// Exclusive prefix of v over a block of NT threads and the block total
// (*tot).  wtot: NT / 64 + 1 doubles of LDS.  Three barriers.
template <int NT>
__device__ __forceinline__ double kpp_block_scan(double v, double *wtot, double *tot) {
  constexpr int NWV = NT / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double s = v;
  for (int off = 1; off < 64; off <<= 1) {
    const double o = __shfl_up(s, off, 64);
    if (lane >= off) s += o;
  }
  double e = __shfl_up(s, 1, 64);
  if (lane == 0) e = 0.0;
  __syncthreads();   // wtot free
  if (lane == 63) wtot[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int k = 0; k < NWV; ++k) {
      const double t = wtot[k];
      wtot[k] = acc;
      acc += t;
    }
    wtot[NWV] = acc;
  }
  __syncthreads();
  *tot = wtot[NWV];
  return wtot[w] + e;
}

// hit = min of the indices `a` >= 0, lastp = max of the indices `l` >= 0
// over the block; indices grow with the lane, so per wave the first (last)
// flagged lane holds the wave's minimum (maximum): one LDS atomic per wave.
__device__ __forceinline__ void kpp_wave_mark(long long a, long long l,
                                              unsigned long long *hit, long long *lastp) {
  const int lane = threadIdx.x & 63;
  const uint64_t ab = __ballot(a >= 0), lb = __ballot(l >= 0);
  if (ab && lane == __builtin_ctzll(ab)) atomicMin(hit, (unsigned long long)a);
  if (lb && lane == 63 - __builtin_clzll(lb)) atomicMax(lastp, l);
}

// The pick of one round by a block of NT threads (all of them call it; all
// get the index): D the n squared distances, T their chunk totals; prev
// is returned when W is not positive.
template <int NT>
__device__ int64_t kpp_pick(const double *__restrict__ D, const double *__restrict__ T,
                            int64_t n, double uj, int64_t prev) {
  constexpr int64_t STAGE = (int64_t)NT * kKppSelPer;
  static_assert(NT >= kKppChunk, "a block covers a chunk");
  __shared__ double wtot[NT / 64 + 1];
  __shared__ unsigned long long hit;   // smallest index above t (~0: none)
  __shared__ long long lastp;          // largest positive index (-1: none)
  __shared__ double hbefore, lbefore;  // running sum before the hit / last
  __shared__ int64_t result;
  const int tid = threadIdx.x;
  const int64_t nch = (n + kKppChunk - 1) / kKppChunk;
  const int64_t nst = (nch + STAGE - 1) / STAGE;
  double v[kKppSelPer];
  double off = 0.0, stot = 0.0;
  auto stage = [&](int64_t st) {   // v, this thread's offset in the stage, the stage total
    const int64_t c0 = st * STAGE + (int64_t)tid * kKppSelPer;
#pragma unroll
    for (int q = 0; q < kKppSelPer; ++q) v[q] = (c0 + q < nch) ? T[c0 + q] : 0.0;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < kKppSelPer; ++q) sum += v[q];
    off = kpp_block_scan<NT>(sum, wtot, &stot);
  };
  // W: the stage totals in order
  double W = 0.0;
  for (int64_t st = 0; st < nst; ++st) {
    stage(st);
    W += stot;
  }
  if (!(W > 0.0)) return prev;   // uniform
  const double t = uj * W;
  // the chunk: first positive chunk total whose running sum exceeds t
  int64_t c = -1, cl = -1;
  double cbefore = 0.0, clbefore = 0.0, base = 0.0;
  for (int64_t st = 0; st < nst; ++st) {
    if (nst > 1) stage(st);
    __syncthreads();
    if (tid == 0) {
      hit = ~0ull;
      lastp = -1;
    }
    __syncthreads();
    double acc = base + off;
    long long mine = -1, myl = -1;
    double mb = 0.0, mlb = 0.0;
#pragma unroll
    for (int q = 0; q < kKppSelPer; ++q) {
      const double nxt = acc + v[q];
      if (v[q] > 0.0) {
        if (mine < 0 && nxt > t) {
          mine = (long long)tid * kKppSelPer + q;
          mb = acc;
        }
        myl = (long long)tid * kKppSelPer + q;
        mlb = acc;
      }
      acc = nxt;
    }
    kpp_wave_mark(mine, myl, &hit, &lastp);
    __syncthreads();
    if (mine >= 0 && (unsigned long long)mine == hit) hbefore = mb;
    if (myl >= 0 && myl == lastp) lbefore = mlb;
    __syncthreads();
    if (hit != ~0ull) {
      c = st * STAGE + (int64_t)hit;
      cbefore = hbefore;
      break;
    }
    if (lastp >= 0) {
      cl = st * STAGE + lastp;
      clbefore = lbefore;
    }
    base += stot;
  }
  if (c < 0) {
    c = cl;
    cbefore = clbefore;
  }
  if (c < 0) return prev;   // a guard: W > 0 has a positive chunk
  // the point: first positive D2 of chunk c whose running sum exceeds t
  const int64_t i0 = c * kKppChunk;
  const double x = (tid < kKppChunk && i0 + tid < n) ? D[i0 + tid] : 0.0;
  double ctot = 0.0;
  const double pre = cbefore + kpp_block_scan<NT>(x, wtot, &ctot);
  __syncthreads();
  if (tid == 0) {
    hit = ~0ull;
    lastp = -1;
  }
  __syncthreads();
  kpp_wave_mark((x > 0.0 && pre + x > t) ? (long long)tid : -1, x > 0.0 ? (long long)tid : -1,
                &hit, &lastp);
  __syncthreads();
  if (tid == 0) {
    const long long p = hit != ~0ull ? (long long)hit : lastp;
    result = p >= 0 ? i0 + p : prev;
  }
  __syncthreads();
  return result;
}

__device__ __forceinline__ double kpp_draw(const double *__restrict__ u, int j) {
  const double uj = u[j];
  return (uj >= 0.0 && uj < 1.0) ? uj : 0.0;  // reported by kpp_first_kernel
}

__global__ __launch_bounds__(kKppSelThreads) void kpp_select_kernel(
    const double *__restrict__ D, const double *__restrict__ T, int64_t n,
    const double *__restrict__ u, int j, int64_t *__restrict__ cidx) {
  const int64_t c = kpp_pick<kKppSelThreads>(D, T, n, kpp_draw(u, j), cidx[j - 1]);
  if (threadIdx.x == 0) cidx[j] = c;
}

// One whole round j >= 1 for clouds of at most kKppFuseChunks chunks:
// every block picks centre j from the distances and chunk totals of round
// j - 1 (Dp, Tp; the same result in every block, written by block 0), then
// forms the distances to it (min with Dp) and the chunk totals of its own
// chunks into Dn, Tn, as kpp_update_kernel does.  Double buffers: no block
// writes what another may still read, and no synchronisation between
// blocks is needed.
constexpr int64_t kKppFuseChunks = (int64_t)kKppUpdThreads * kKppSelPer;
__global__ __launch_bounds__(kKppUpdThreads) void kpp_round_kernel(
    const float *__restrict__ pts, int64_t n, const double *__restrict__ u, int j,
    int64_t *__restrict__ cidx, const double *__restrict__ Dp, const double *__restrict__ Tp,
    double *__restrict__ Dn, double *__restrict__ Tn, int64_t nch) {
  __shared__ double sh[kKppUpdChunks * kKppRow];
  const int64_t c = kpp_pick<kKppUpdThreads>(Dp, Tp, n, kpp_draw(u, j), cidx[j - 1]);
  if (blockIdx.x == 0 && threadIdx.x == 0) cidx[j] = c;
  const double c0 = pts[3 * c], c1 = pts[3 * c + 1], c2 = pts[3 * c + 2];
  const int64_t base = (int64_t)blockIdx.x * kKppUpdChunks * kKppChunk;
  constexpr int PER = kKppUpdChunks * kKppChunk / kKppUpdThreads;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int l = q * kKppUpdThreads + threadIdx.x;
    const int64_t i = base + l;
    double v = 0.0;  // past the end: 0, which leaves the running sums as they are
    if (i < n) {
      const double d = kpp_d2(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], c0, c1, c2);
      const double o = Dp[i];
      v = d < o ? d : o;
      Dn[i] = v;
    }
    sh[(l / kKppChunk) * kKppRow + (l % kKppChunk)] = v;
  }
  __syncthreads();
  const int64_t ch = (int64_t)blockIdx.x * kKppUpdChunks + threadIdx.x;
  if (threadIdx.x < kKppUpdChunks && ch < nch) {
    const double *a = sh + threadIdx.x * kKppRow;
    double s = 0.0;
    for (int k0 = 0; k0 < kKppChunk; k0 += 16) {
      double e[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) e[k] = a[k0 + k];
#pragma unroll
      for (int k = 0; k < 16; ++k) s += e[k];
    }
    Tn[ch] = s;
  }
}

// Non-finite coordinates (for a call that forms no distances otherwise).
__global__ __launch_bounds__(256) void kpp_check_kernel(const float *__restrict__ pts,
                                                        int64_t n, uint32_t *status) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && (!isfinite(pts[3 * i]) || !isfinite(pts[3 * i + 1]) || !isfinite(pts[3 * i + 2])))
    set_status(status, kStNonFinite);
}

// label_i = the nearest of the K centres (lowest index on ties).
__global__ __launch_bounds__(kKppLabelThreads) void kpp_label_kernel(
    const float *__restrict__ pts, int64_t n, const int64_t *__restrict__ cidx, int K,
    int32_t *__restrict__ labels, uint32_t *status) {
  extern __shared__ __align__(16) unsigned char kpp_smem[];
  double *cs = reinterpret_cast<double *>(kpp_smem);  // K x 3
  for (int k = threadIdx.x; k < K; k += kKppLabelThreads) {
    const int64_t c = cidx[k];
    cs[3 * k] = pts[3 * c];
    cs[3 * k + 1] = pts[3 * c + 1];
    cs[3 * k + 2] = pts[3 * c + 2];
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kKppLabelThreads + threadIdx.x;
  if (i >= n) return;
  const float f0 = pts[3 * i], f1 = pts[3 * i + 1], f2 = pts[3 * i + 2];
  if (!isfinite(f0) || !isfinite(f1) || !isfinite(f2)) set_status(status, kStNonFinite);
  const double x0 = f0, x1 = f1, x2 = f2;
  double best = kpp_d2(x0, x1, x2, cs[0], cs[1], cs[2]);
  int l = 0;
  for (int k = 1; k < K; ++k) {
    const double d = kpp_d2(x0, x1, x2, cs[3 * k], cs[3 * k + 1], cs[3 * k + 2]);
    if (d < best) {
      best = d;
      l = k;
    }
  }
  labels[i] = l;
}

}  // namespace gmm_dev
