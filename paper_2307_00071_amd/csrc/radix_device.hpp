// Stable LSD radix sort of (32-bit key, 32-bit value) pairs by one 8-bit
// digit per pass, and the block scans it is built from (device code).
//
// A pass is three launches over nblk = ceil(n / kSortChunk) blocks:
//   radix_hist_kernel     digit counts of each block's chunk;
//   radix_scan_kernel     per digit (one block each), the exclusive prefix of
//                         its counts over the blocks, and the digit total;
//   radix_scatter_kernel  a stable scatter: digit starts from the totals,
//                         ranks within a block from wave ballots, waves and
//                         rounds in item order.
// Keys wider than 32 bits are sorted word by word, least significant first,
// the next word gathered through the values in between.  No step clears
// memory with a memset, so a sequence of passes can be captured in a graph.
// Internal linkage: every translation unit that includes this header gets
// its own copy of the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmm_dev {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;                           // per thread and pass
constexpr int kSortChunk = kSortThreads * kSortItems;   // items per block

// Digit counts of one block's chunk: hist[digit * nblk + block].
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(
    const unsigned *__restrict__ keys, int64_t npad, int shift,
    unsigned *__restrict__ hist, int nblk) {
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t i = base + it * kSortThreads + threadIdx.x;
    if (i < npad) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Per-digit scan: block d turns hist[d * nblk .. (d + 1) * nblk) into its
// exclusive prefix (in place) and writes the digit total dtot[d].  Each
// thread takes a contiguous run of kScanPer counts; runs are scanned within
// a wave by shuffles and across the block's waves by wave 0.
constexpr int kScanPer = 8;

__device__ inline unsigned wave_inclusive_scan(unsigned v, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread over a 256-thread block (four
// waves); *total gets the block sum.  Two barriers.
__device__ inline unsigned block_exclusive_scan256(unsigned v, unsigned *wsum,
                                                   unsigned *total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned inc = wave_inclusive_scan(v, lane);
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  unsigned off = 0, tot = 0;
#pragma unroll
  for (int j = 0; j < kSortThreads / 64; ++j) {
    const unsigned w = wsum[j];
    off += j < wv ? w : 0u;
    tot += w;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ __launch_bounds__(kSortThreads) void radix_scan_kernel(
    unsigned *__restrict__ hist, int nblk, unsigned *__restrict__ dtot) {
  __shared__ unsigned wsum[kSortThreads / 64];
  unsigned *h = hist + (size_t)blockIdx.x * nblk;
  unsigned carry = 0;
  for (int base = 0; base < nblk; base += kSortThreads * kScanPer) {
    const int a = base + threadIdx.x * kScanPer;
    unsigned v[kScanPer];
    unsigned s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      v[j] = (a + j < nblk) ? h[a + j] : 0u;
      s += v[j];
    }
    unsigned tot = 0;
    unsigned run = carry + block_exclusive_scan256(s, wsum, &tot);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      if (a + j < nblk) h[a + j] = run;
      run += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Stable scatter of one block's chunk by the digit at `shift`.  Items are
// taken in rounds of one per thread; within a round an item's rank among
// equal digits comes from wave ballots (lower lanes first) and the counts
// of the lower waves, after every item of the earlier rounds.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const unsigned *__restrict__ kin, const unsigned *__restrict__ vin,
    int64_t npad, int shift, const unsigned *__restrict__ off, int nblk,
    const unsigned *__restrict__ dtot, unsigned *__restrict__ kout,
    unsigned *__restrict__ vout) {
  constexpr int W = kSortThreads / 64;
  __shared__ unsigned run[256];
  __shared__ unsigned wc[W][256];
  __shared__ unsigned wsum[W];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  unsigned all = 0;
  const unsigned dstart = block_exclusive_scan256(dtot[tid], wsum, &all);
  run[tid] = dstart + off[(size_t)tid * nblk + blockIdx.x];
  for (int v = 0; v < W; ++v) wc[v][tid] = 0u;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t i = base + it * kSortThreads + tid;
    const bool ok = i < npad;
    const unsigned k = ok ? kin[i] : 0u;
    const unsigned d = (k >> shift) & 255u;
    uint64_t pm = __ballot(ok);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t bm = __ballot((d >> bit) & 1u);
      pm &= ((d >> bit) & 1u) ? bm : ~bm;
    }
    const unsigned rank = (unsigned)__popcll(pm & lt);
    const bool last = ((pm >> lane) >> 1) == 0ull;
    if (ok && last) wc[w][d] = rank + 1u;
    __syncthreads();
    if (ok) {
      unsigned pos = run[d] + rank;
      for (int v = 0; v < w; ++v) pos += wc[v][d];
      kout[pos] = k;
      vout[pos] = vin[i];
    }
    __syncthreads();
    unsigned add = 0u;
    for (int v = 0; v < W; ++v) {
      add += wc[v][tid];
      wc[v][tid] = 0u;
    }
    run[tid] += add;
    __syncthreads();
  }
}

}  // namespace
}  // namespace gmm_dev
