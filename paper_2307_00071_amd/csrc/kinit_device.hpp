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
// sequential within chunks of kKppChunk points, chunk totals sequential
// within groups of kKppGroup chunks, group totals sequential.  The search
// walks the groups, then the chunks of the chosen group, then the points of
// the chosen chunk, each time against what is left of u W; where rounding
// leaves no running sum above it, the last positive entry is taken.
// Squared distances are ((dx^2 + dy^2) + dz^2) in double with every
// operation rounded on its own (no contraction).
//
// Per round j >= 1: kpp_update_kernel (D2 with centre j - 1, chunk totals)
// and kpp_select_kernel (one block: group totals, W, the search).  The
// update streams 28 B per point per round (the point, D2 read and
// written); the select kernel is a short chain of dependent reads and
// serial sums; neither does enough arithmetic to meet a compute roofline.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmm_dev {

constexpr int kKppChunk = 256;      // points per chunk (running-sum order)
constexpr int kKppGroup = 64;       // chunks per group
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

// Sequential total of the chunk totals of group g (16 loads in flight).
__device__ __forceinline__ double kpp_group_total(const double *__restrict__ T, int64_t nch,
                                                  int64_t g) {
  const int64_t lo = g * kKppGroup;
  const int cnt = (int)(nch - lo < kKppGroup ? nch - lo : kKppGroup);
  double s = 0.0;
  int c = 0;
  for (; c + 16 <= cnt; c += 16) {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = T[lo + c + q];
#pragma unroll
    for (int q = 0; q < 16; ++q) s += v[q];
  }
  for (; c < cnt; ++c) s += T[lo + c];
  return s;
}

// Result of one walk over an array.
struct KppWalk {
  double total;        // running sum at the end
  double before;       // running sum before `idx`
  long long idx;       // first index whose running sum exceeds t, else the
                       // last positive entry, else -1
  long long hit, last; // block reductions (LDS)
};

// out->hit = min index of the block's threads with `above`, out->last = max
// index with `positive`: per wave a ballot, then one LDS atomic per wave.
__device__ __forceinline__ void kpp_mark(bool above, bool positive, KppWalk *out) {
  const uint64_t a = __ballot(above), p = __ballot(positive);
  if ((threadIdx.x & 63) == 0) {
    const int wbase = threadIdx.x & ~63;
    if (a) atomicMin(reinterpret_cast<unsigned long long *>(&out->hit),
                     (unsigned long long)(wbase + __builtin_ctzll(a)));
    if (p) atomicMax(&out->last, (long long)(wbase + 63 - __builtin_clzll(p)));
  }
}

// v[0..m) in order.  Per stage of kKppSelThreads entries thread 0 forms the
// running sums sequentially (only the dependent additions are serial; the
// values are read 16 at a time) into `pre`; then every thread compares
// its own entry with t, and the first index above t (or the last positive
// entry) is found by block-wide minimum / maximum.  Same values and the
// same choice as a single sequential walk.
__device__ void kpp_walk(const double *__restrict__ v, int64_t m, bool search, double t,
                         double *stage, double *pre, KppWalk *out) {
  double acc = 0.0;  // thread 0: running sum before this stage
  bool found = false;
  for (int64_t base = 0; base < m; base += kKppSelThreads) {
    const int cnt = (int)(m - base < kKppSelThreads ? m - base : kKppSelThreads);
    __syncthreads();  // stage and pre free; out->hit / out->last reset
    if (threadIdx.x == 0) {
      out->hit = -1;
      out->last = -1;
    }
    // zeros past the end leave the running sums unchanged and are never
    // above t or positive, so the walk needs no bounds inside
    stage[threadIdx.x] = threadIdx.x < cnt ? v[base + threadIdx.x] : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = acc;
      for (int k0 = 0; k0 < cnt; k0 += 16) {
        double e[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) e[q] = stage[k0 + q];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          a = a + e[q];
          pre[k0 + q] = a;
        }
      }
      pre[kKppSelThreads] = acc;  // running sum before the stage
      acc = a;
    }
    __syncthreads();
    kpp_mark(threadIdx.x < cnt && search && pre[threadIdx.x] > t,
             threadIdx.x < cnt && stage[threadIdx.x] > 0.0, out);
    __syncthreads();
    // hit: -1 is the largest unsigned value, so atomicMin keeps any real index
    if (out->hit >= 0 && out->hit < cnt) {
      if (threadIdx.x == 0) {
        const int h = (int)out->hit;
        out->idx = base + h;
        out->before = h > 0 ? pre[h - 1] : pre[kKppSelThreads];
        out->total = acc;
      }
      found = true;
      break;
    }
    if (threadIdx.x == 0 && out->last >= 0) {
      const int l = (int)out->last;
      out->idx = base + l;  // last positive so far
      out->before = l > 0 ? pre[l - 1] : pre[kKppSelThreads];
    }
  }
  if (!found && threadIdx.x == 0) out->total = acc;
  __syncthreads();
}

// W and the group search in one pass when the group totals fit one stage:
// the running sums of stage[0..m) (m <= kKppSelThreads) serially into pre,
// W = the last, t = uj W, then the first running sum above t (else the
// last positive entry) in parallel.  out->idx = -2 when W is not positive.
__device__ void kpp_draw_walk(int m, double uj, double *stage, double *pre, KppWalk *out) {
  // stage[0..kKppSelThreads) holds v, zeros past m (see kpp_walk)
  if (threadIdx.x == 0) {
    out->hit = -1;
    out->last = -1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int k0 = 0; k0 < m; k0 += 16) {
      double e[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) e[q] = stage[k0 + q];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        a = a + e[q];
        pre[k0 + q] = a;
      }
    }
    out->total = a;
  }
  __syncthreads();
  const double W = out->total;
  if (!(W > 0.0)) {
    if (threadIdx.x == 0) out->idx = -2;
    __syncthreads();
    return;
  }
  const double t = uj * W;
  kpp_mark(threadIdx.x < m && pre[threadIdx.x] > t, threadIdx.x < m && stage[threadIdx.x] > 0.0,
           out);
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long h = out->hit >= 0 ? out->hit : out->last;
    out->idx = h;
    out->before = h > 0 ? pre[h - 1] : 0.0;
  }
  __syncthreads();
}

// Centre j >= 1 from the chunk totals T (group totals formed here; U is
// scratch for more than kKppSelThreads groups) and the per-point D2.  One
// block.
__global__ __launch_bounds__(kKppSelThreads) void kpp_select_kernel(
    const double *__restrict__ D, const double *__restrict__ T, double *__restrict__ U,
    int64_t n, const double *__restrict__ u, int j, int64_t *__restrict__ cidx) {
  __shared__ double stage[kKppSelThreads];
  __shared__ double pre[kKppSelThreads + 1];
  __shared__ KppWalk w;
  const int64_t nch = (n + kKppChunk - 1) / kKppChunk;
  const int64_t ngr = (nch + kKppGroup - 1) / kKppGroup;
  double uj = u[j];
  if (!(uj >= 0.0 && uj < 1.0)) uj = 0.0;  // reported by kpp_first_kernel
  double t;
  if (ngr <= kKppSelThreads) {
    stage[threadIdx.x] = threadIdx.x < ngr ? kpp_group_total(T, nch, threadIdx.x) : 0.0;
    kpp_draw_walk((int)ngr, uj, stage, pre, &w);
    if (w.idx == -2) {
      if (threadIdx.x == 0) cidx[j] = cidx[j - 1];
      return;
    }
    t = uj * w.total;
  } else {
    for (int64_t g = threadIdx.x; g < ngr; g += kKppSelThreads) U[g] = kpp_group_total(T, nch, g);
    if (threadIdx.x == 0) w.idx = -1;
    __syncthreads();
    kpp_walk(U, ngr, false, 0.0, stage, pre, &w);
    const double W = w.total;
    if (!(W > 0.0)) {
      if (threadIdx.x == 0) cidx[j] = cidx[j - 1];
      return;
    }
    t = uj * W;
    __syncthreads();
    if (threadIdx.x == 0) w.idx = -1;
    __syncthreads();
    kpp_walk(U, ngr, true, t, stage, pre, &w);
  }
  // (an index < 0 cannot follow W > 0; kept as a guard for the indexing)
  if (w.idx < 0) {
    if (threadIdx.x == 0) cidx[j] = cidx[j - 1];
    return;
  }
  const int64_t g = w.idx;
  const double t1 = t - w.before;
  const int64_t clo = g * kKppGroup;
  const int64_t cm = nch - clo < kKppGroup ? nch - clo : kKppGroup;
  __syncthreads();
  if (threadIdx.x == 0) w.idx = -1;
  __syncthreads();
  kpp_walk(T + clo, cm, true, t1, stage, pre, &w);
  if (w.idx < 0) {
    if (threadIdx.x == 0) cidx[j] = cidx[j - 1];
    return;
  }
  const int64_t c = clo + w.idx;
  const double t2 = t1 - w.before;
  const int64_t ilo = c * kKppChunk;
  const int64_t im = n - ilo < kKppChunk ? n - ilo : kKppChunk;
  __syncthreads();
  if (threadIdx.x == 0) w.idx = -1;
  __syncthreads();
  kpp_walk(D + ilo, im, true, t2, stage, pre, &w);
  if (threadIdx.x == 0) cidx[j] = w.idx < 0 ? cidx[j - 1] : ilo + w.idx;
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
