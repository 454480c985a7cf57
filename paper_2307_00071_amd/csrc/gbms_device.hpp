// Mean shift with a flat kernel over binned seeds (device code, included by
// gbms.hip): the estimate of the number of mixture components that precedes
// k-means++ seeding and EM (the paper, Sec. V "Gaussian Blurring Mean Shift"
// and the information-flow figure: bandwidth + point cloud -> K).
//
// Seeds are the centres b h of the occupied bins b = rint(x / h) (Comaniciu
// and Meer's binned estimator); a seed moves to the mean of the points within
// distance h of it until the move is at most 1e-3 h or the iteration cap is
// reached; its weight is the size of that last neighbourhood.  Modes are then
// merged: in the order (weight descending, coordinates descending, seed
// ascending) a mode still kept removes every later mode within h.
//
// GPU design:
//   * a uniform grid of cell side h, the cells being the bins themselves:
//     the points are sorted by the 64-bit packed bin key (stable LSD radix
//     sort, radix_device.hpp), the occupied cells are the runs of equal keys
//     (so the seeds come out in lexicographic bin order) and an open-
//     addressing hash table maps a key to its cell;
//   * one wave per seed: a ball of radius h around s overlaps at most four
//     cells per axis, and cell k goes to the slot given by k mod 4 on every
//     axis (4^D slots, lane = slot mod 64), so the cell that holds a point
//     reaches the same lane whatever s is: the neighbourhood sum is then a
//     function of the neighbourhood alone (each lane adds its cells' points
//     in sorted order, rounds in order, then a fixed DPP reduction: within
//     each 16-lane row, then the rows in order), and seeds
//     that reach the same neighbourhood get bitwise the same mean;
//   * the merge never sorts the modes: mode i is kept iff no kept mode that
//     precedes it lies within h, so it needs only the predecessors within h
//     (a second grid, over the modes).  Rounds decide, in place, every mode
//     whose predecessors within h are all decided; each round decides at
//     least the first undecided mode of the order, so the rounds end.
// All arithmetic that decides a neighbourhood, a bin, a stop or a merge is
// FP64 with every product and sum rounded on its own (no contraction), in the
// order ((d0^2 + d1^2) + d2^2) + d3^2.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "radix_device.hpp"
#include "wave_f64.hpp"

#pragma clang fp contract(off)

namespace gbms_dev {

using namespace gmm_wave;

using gmm_dev::kSortChunk;
using gmm_dev::kSortItems;
using gmm_dev::kSortThreads;

constexpr int kMsThreads = 256;
constexpr int kMsWaves = kMsThreads / 64;   // seeds (or modes) per block
constexpr uint64_t kNoKey = ~0ull;          // empty hash slot; no real key has it
constexpr int kRoundBatch = 16;             // merge rounds per host check

// device status bits
constexpr uint32_t kMsNonFinite = 1u;
constexpr uint32_t kMsRange = 2u;

__device__ inline void ms_set_status(uint32_t *st, uint32_t bit) { atomicOr(st, bit); }

// Bin keys: D fields of kBits[D] bits, the first coordinate most
// significant, each holding b + 2^(bits - 1) with |b| <= 2^(bits - 1) - 2,
// so that key order is the lexicographic order of the bins and no key is
// all ones.
template <int D> struct KeyBits;
template <> struct KeyBits<3> { static constexpr int v = 21; };
template <> struct KeyBits<4> { static constexpr int v = 16; };

template <int D>
__device__ __forceinline__ int64_t bin_limit() {
  return (int64_t(1) << (KeyBits<D>::v - 1)) - 2;
}

template <int D>
__device__ __forceinline__ bool pack_key(const int64_t *b, uint64_t *key) {
  constexpr int B = KeyBits<D>::v;
  const int64_t lim = bin_limit<D>();
  uint64_t k = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    if (b[j] < -lim || b[j] > lim) return false;
    k = (k << B) | (uint64_t)(b[j] + (int64_t(1) << (B - 1)));
  }
  *key = k;
  return true;
}

template <int D>
__device__ __forceinline__ void unpack_key(uint64_t key, int64_t *b) {
  constexpr int B = KeyBits<D>::v;
#pragma unroll
  for (int j = D - 1; j >= 0; --j) {
    b[j] = (int64_t)(key & ((uint64_t(1) << B) - 1)) - (int64_t(1) << (B - 1));
    key >>= B;
  }
}

// SplitMix64's output mix (Steele, Lea and Flood 2014) as the hash.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xbf58476d1ce4e5b9ull;
  z ^= z >> 27;
  z *= 0x94d049bb133111ebull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ int hash_find(const uint64_t *__restrict__ hk,
                                         const int *__restrict__ hv, uint64_t mask,
                                         uint64_t key) {
  uint64_t s = mix64(key) & mask;
  for (;;) {
    const uint64_t k = hk[s];
    if (k == key) return hv[s];
    if (k == kNoKey) return -1;
    s = (s + 1) & mask;
  }
}

// ((d0^2 + d1^2) + d2^2) (+ d3^2), each operation rounded on its own.
template <int D>
__device__ __forceinline__ double sq_norm(const double *d) {
  double q = d[0] * d[0] + d[1] * d[1];
#pragma unroll
  for (int j = 2; j < D; ++j) q = q + d[j] * d[j];
  return q;
}

// ------------------------------------------------------------ point keys
// Key of point i from b_j = rint(x_j / h) in FP64; vals[i] = i.
template <int D>
__global__ __launch_bounds__(kSortThreads) void ms_point_key_kernel(
    const float *__restrict__ pts, int64_t n, double h, unsigned *__restrict__ klo,
    unsigned *__restrict__ khi, unsigned *__restrict__ vals, uint32_t *__restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
  if (i >= n) return;
  int64_t b[D];
  bool fin = true;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const double x = (double)pts[i * D + j];
    fin = fin && isfinite(x);
    const double r = rint(x / h);
    b[j] = (fabs(r) < 4.0e18) ? (int64_t)r : 0;
  }
  uint64_t key = 0;
  if (!fin) {
    ms_set_status(status, kMsNonFinite);
  } else if (!pack_key<D>(b, &key)) {
    ms_set_status(status, kMsRange);
  }
  klo[i] = (unsigned)key;
  khi[i] = (unsigned)(key >> 32);
  vals[i] = (unsigned)i;
}

// Key of mode i (bins of the mode grid) for i < n items; all ones for a
// dropped seed and for the items past the seed count *nsp.
template <int D>
__global__ __launch_bounds__(kSortThreads) void ms_mode_key_kernel(
    const double *__restrict__ mode, const int *__restrict__ weight,
    const int *__restrict__ nsp, int64_t n, double h, unsigned *__restrict__ klo,
    unsigned *__restrict__ khi, unsigned *__restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
  if (i >= n) return;
  uint64_t key = kNoKey;
  if (i < *nsp && weight[i] > 0) {
    int64_t b[D];
#pragma unroll
    for (int j = 0; j < D; ++j) b[j] = (int64_t)rint(mode[(size_t)i * D + j] / h);
    if (!pack_key<D>(b, &key)) key = kNoKey;   // cannot happen: modes are means of points
  }
  klo[i] = (unsigned)key;
  khi[i] = (unsigned)(key >> 32);
  vals[i] = (unsigned)i;
}

// out[i] = in[perm[i]] (32-bit words)
__global__ __launch_bounds__(kSortThreads) void ms_gather_u32_kernel(
    const unsigned *__restrict__ in, const unsigned *__restrict__ perm,
    const int *__restrict__ np, int64_t nmax, unsigned *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
  const int64_t n = np ? (int64_t)*np : nmax;
  if (i < n) out[i] = in[perm[i]];
}

// Sorted 64-bit keys and, for the points, the sorted float4 copies.
template <int D>
__global__ __launch_bounds__(kSortThreads) void ms_sorted_kernel(
    const unsigned *__restrict__ klo, const unsigned *__restrict__ khi,
    const unsigned *__restrict__ perm, const float *__restrict__ pts,
    const int *__restrict__ np, int64_t nmax, uint64_t *__restrict__ keys,
    float4 *__restrict__ ptsS) {
  const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
  const int64_t n = np ? (int64_t)*np : nmax;
  if (i >= n) return;
  const unsigned p = perm[i];
  keys[i] = ((uint64_t)khi[p] << 32) | klo[p];
  if (ptsS) {
    const float *x = pts + (size_t)p * D;
    ptsS[i] = make_float4(x[0], x[1], x[2], D == 4 ? x[3] : 0.0f);
  }
}

// ------------------------------------------------- flags and their scan
// Two flag kinds over n items: a new run of sorted keys (FLAG_CELL), or a
// kept mode (FLAG_KEPT).  Each block takes a chunk of kSortChunk items,
// thread t the kSortItems consecutive items from t kSortItems on.
enum { FLAG_CELL = 0, FLAG_KEPT = 1 };

template <int KIND>
__device__ __forceinline__ bool item_flag(const uint64_t *keys, const int *status, int64_t i) {
  if (KIND == FLAG_CELL) return i == 0 || keys[i] != keys[i - 1];
  return status[i] == 1;
}

template <int KIND>
__global__ __launch_bounds__(kSortThreads) void ms_flag_count_kernel(
    const uint64_t *__restrict__ keys, const int *__restrict__ status,
    const int *__restrict__ np, int64_t nmax, unsigned *__restrict__ bsum) {
  __shared__ unsigned wsum[kSortThreads / 64];
  const int64_t n = np ? (int64_t)*np : nmax;
  const int64_t base = (int64_t)blockIdx.x * kSortChunk + (int64_t)threadIdx.x * kSortItems;
  unsigned c = 0;
#pragma unroll
  for (int u = 0; u < kSortItems; ++u) {
    const int64_t i = base + u;
    if (i < n && item_flag<KIND>(keys, status, i)) ++c;
  }
  unsigned tot = 0;
  (void)gmm_dev::block_exclusive_scan256(c, wsum, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// FLAG_CELL: start[cell] = first sorted index of the cell, ckey[cell] = its
// key.  FLAG_KEPT: the kept modes in seed order into (out_mode, out_w).
// boff = the exclusive scan of the block counts.
template <int KIND, int D>
__global__ __launch_bounds__(kSortThreads) void ms_flag_write_kernel(
    const uint64_t *__restrict__ keys, const int *__restrict__ status,
    const int *__restrict__ np, int64_t nmax, const unsigned *__restrict__ boff,
    int *__restrict__ start, uint64_t *__restrict__ ckey,
    const double *__restrict__ mode, const int *__restrict__ weight,
    double *__restrict__ out_mode, long long *__restrict__ out_w, int64_t out_cap) {
  __shared__ unsigned wsum[kSortThreads / 64];
  const int64_t n = np ? (int64_t)*np : nmax;
  const int64_t base = (int64_t)blockIdx.x * kSortChunk + (int64_t)threadIdx.x * kSortItems;
  unsigned c = 0;
  bool f[kSortItems];
#pragma unroll
  for (int u = 0; u < kSortItems; ++u) {
    const int64_t i = base + u;
    f[u] = i < n && item_flag<KIND>(keys, status, i);
    c += f[u] ? 1u : 0u;
  }
  unsigned tot = 0;
  unsigned pos = boff[blockIdx.x] + gmm_dev::block_exclusive_scan256(c, wsum, &tot);
#pragma unroll
  for (int u = 0; u < kSortItems; ++u) {
    if (!f[u]) continue;
    const int64_t i = base + u;
    if (KIND == FLAG_CELL) {
      start[pos] = (int)i;
      ckey[pos] = keys[i];
    } else if ((int64_t)pos < out_cap) {
#pragma unroll
      for (int j = 0; j < D; ++j) out_mode[(size_t)pos * D + j] = mode[(size_t)i * D + j];
      if (out_w) out_w[pos] = (long long)weight[i];
    }
    ++pos;
  }
}

// start[ncells] = n; the cell count to *count.
__global__ void ms_cells_end_kernel(const unsigned *__restrict__ dtot,
                                    const int *__restrict__ np, int64_t nmax,
                                    int *__restrict__ start, int *__restrict__ count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int nc = (int)dtot[0];
  start[nc] = np ? *np : (int)nmax;
  *count = nc;
}

// ---------------------------------------------------------------- hashing
__global__ __launch_bounds__(kSortThreads) void ms_hash_clear_kernel(
    uint64_t *__restrict__ hk, uint64_t cap) {
  const uint64_t i = (uint64_t)blockIdx.x * kSortThreads + threadIdx.x;
  if (i < cap) hk[i] = kNoKey;
}

// Cell c's key into the table (the all-ones key of dropped seeds is not).
__global__ __launch_bounds__(kSortThreads) void ms_hash_insert_kernel(
    const uint64_t *__restrict__ ckey, const int *__restrict__ ncp,
    uint64_t *__restrict__ hk, int *__restrict__ hv, uint64_t mask) {
  const int c = blockIdx.x * kSortThreads + threadIdx.x;
  if (c >= *ncp) return;
  const uint64_t key = ckey[c];
  if (key == kNoKey) return;
  uint64_t s = mix64(key) & mask;
  for (;;) {
    const unsigned long long prev =
        atomicCAS(reinterpret_cast<unsigned long long *>(hk + s),
                  (unsigned long long)kNoKey, (unsigned long long)key);
    if (prev == (unsigned long long)kNoKey) {
      hv[s] = c;
      return;
    }
    s = (s + 1) & mask;
  }
}

// ------------------------------------------------------- the grid query
// Cells whose bins can hold a point within h of s: per axis the bins from
// ceil(s/h - 1.5) to floor(s/h + 1.5), widened by 1e-7 (rounding of x / h
// and of the distance test); at most four per axis.  Slot u (4^D of them)
// stands for the cell whose bin is congruent to the base-4 digits of u on
// every axis; the slot is skipped when that bin is outside the range or its
// box is farther than h from s.
template <int D>
struct GridQuery {
  double t[D];
  int lo[D], nr[D];
  __device__ __forceinline__ void init(const double *s, double h) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      t[j] = s[j] / h;
      lo[j] = (int)ceil(t[j] - 1.5 - 1e-7);
      nr[j] = (int)floor(t[j] + 1.5 + 1e-7) - lo[j] + 1;
    }
  }
  __device__ __forceinline__ bool slot_key(int u, uint64_t *key) const {
    int64_t k[D];
    double g2 = 0.0;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int r = (u >> (2 * (D - 1 - j))) & 3;
      const int off = (r - lo[j]) & 3;
      k[j] = (int64_t)lo[j] + off;
      ok = ok && off < nr[j];
      const double g = fabs(t[j] - (double)k[j]) - 0.5;
      if (g > 0.0) g2 = g2 + g * g;
    }
    ok = ok && g2 <= 1.0 + 1e-6;
    return ok && pack_key<D>(k, key);
  }
};

// -------------------------------------------------------------- mean shift
// Cells with at most kMsSerial points are walked by the lane that owns their
// slot; larger cells by the whole wave (point p of a cell starting at b goes
// to lane (p - b) mod 64), one cell after another in slot order.  Every lane
// therefore sums its points in an order fixed by the cells alone: the mean
// of an iterate depends only on the set of points within h of it.
constexpr int kMsSerial = 16;
constexpr int kMsBlockSeeds = 16384;   // at most this many seeds: four waves per seed

template <int D>
__device__ __forceinline__ void ms_take(const float4 &x, bool ok, const double *s, double h2,
                                        double *acc, int &in) {
  const double xv[4] = {(double)x.x, (double)x.y, (double)x.z, (double)x.w};
  double d[D];
#pragma unroll
  for (int j = 0; j < D; ++j) d[j] = xv[j] - s[j];
  if (ok && sq_norm<D>(d) <= h2) {
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = acc[j] + xv[j];
    ++in;
  }
}

// One wave per seed (a cell, in sorted order = lexicographic bin order):
// mode, weight (the last neighbourhood's size; 0 = dropped) and the
// iteration count of the oracle's loop.
template <int D>
__global__ __launch_bounds__(kMsThreads) void ms_shift_kernel(
    const float4 *__restrict__ ptsS, const int *__restrict__ cstart,
    const uint64_t *__restrict__ ckey, const int *__restrict__ ncp,
    const uint64_t *__restrict__ hk, const int *__restrict__ hv, uint64_t mask,
    double h, int max_iter, double *__restrict__ mode, int *__restrict__ weight,
    int *__restrict__ iters, int *__restrict__ max_it, int thr) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * kMsWaves + (threadIdx.x >> 6);
  const int ncells = *ncp;
  if (ncells <= thr) return;   // few seeds: ms_shift4_kernel takes them
  if (c >= ncells) return;     // uniform per wave
  double s[D];
  {
    int64_t b[D];
    unpack_key<D>(ckey[c], b);
#pragma unroll
    for (int j = 0; j < D; ++j) s[j] = (double)b[j] * h;
  }
  const double h2 = h * h;
  const double stop = 1e-3 * h;
  int it = 0, cnt = 0;
  for (;;) {
    GridQuery<D> g;
    g.init(s, h);
    double acc[D];
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = 0.0;
    int in = 0;
    for (int u0 = 0; u0 < (1 << (2 * D)); u0 += 64) {
      int b = 0, e = 0;
      uint64_t key;
      if (g.slot_key(u0 + lane, &key)) {
        const int id = hash_find(hk, hv, mask, key);
        if (id >= 0) {
          b = cstart[id];
          e = cstart[id + 1];
        }
      }
      const bool wide = e - b > kMsSerial;
      if (!wide) {
        for (int p0 = b; p0 < e; p0 += 4) {
          float4 x[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) x[k] = ptsS[min(p0 + k, e - 1)];
#pragma unroll
          for (int k = 0; k < 4; ++k) ms_take<D>(x[k], p0 + k < e, s, h2, acc, in);
        }
      }
      uint64_t big = __ballot(wide);
      while (big) {
        const int o = __builtin_ctzll(big);
        big &= big - 1;
        const int cb = __builtin_amdgcn_readlane(b, o);
        const int ce = __builtin_amdgcn_readlane(e, o);
        for (int p0 = cb + lane; p0 < ce; p0 += 256) {
          float4 x[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) x[k] = ptsS[min(p0 + 64 * k, ce - 1)];
#pragma unroll
          for (int k = 0; k < 4; ++k) ms_take<D>(x[k], p0 + 64 * k < ce, s, h2, acc, in);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = wave_sum_f64(acc[j]);
    in = wave_sum_i32(in);
    if (in == 0) break;   // uniform: every lane holds the same sums
    cnt = in;
    double d[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double v = acc[j] / (double)in;
      d[j] = v - s[j];
      s[j] = v;
    }
    if (sqrt(sq_norm<D>(d)) <= stop || it == max_iter) break;
    ++it;
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < D; ++j) mode[(size_t)c * D + j] = s[j];
    weight[c] = cnt;
    iters[c] = it;
    atomicMax(max_it, it);
  }
}

// The same shift with the four waves of a block on one seed, for calls with
// at most `thr` seeds (few seeds, large neighbourhoods: the time is the
// slowest seed's chain of iterations).  Wave w probes the slots of rounds
// w, w + 4, ... and walks their small cells lane by lane; the wide cells of
// every round go to LDS in slot order and all 256 lanes walk them one
// after another (point b + k to thread k mod 256); the four wave sums are
// added in wave order.  Every lane's order is again fixed by the cells
// alone.  Two barriers per iteration.
template <int D>
__global__ __launch_bounds__(kMsThreads) void ms_shift4_kernel(
    const float4 *__restrict__ ptsS, const int *__restrict__ cstart,
    const uint64_t *__restrict__ ckey, const int *__restrict__ ncp,
    const uint64_t *__restrict__ hk, const int *__restrict__ hv, uint64_t mask,
    double h, int max_iter, double *__restrict__ mode, int *__restrict__ weight,
    int *__restrict__ iters, int *__restrict__ max_it, int thr) {
  constexpr int NR = (1 << (2 * D)) / 64;   // rounds of 64 slots
  constexpr int NW = kMsThreads / 64;
  __shared__ int wb[NR][64], we[NR][64];    // wide cells of each round, slot order
  __shared__ int wn[NR];
  __shared__ double part[NW][D + 1];
  const int ncells = *ncp;
  if (ncells > thr) return;                 // many seeds: ms_shift_kernel takes them
  const int c = blockIdx.x;
  if (c >= ncells) return;                  // uniform per block
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double s[D];
  {
    int64_t b[D];
    unpack_key<D>(ckey[c], b);
#pragma unroll
    for (int j = 0; j < D; ++j) s[j] = (double)b[j] * h;
  }
  const double h2 = h * h;
  const double stop = 1e-3 * h;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int it = 0, cnt = 0;
  for (;;) {
    GridQuery<D> g;
    g.init(s, h);
    double acc[D];
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = 0.0;
    int in = 0;
    for (int r = w; r < NR; r += NW) {
      int b = 0, e = 0;
      uint64_t key;
      if (g.slot_key(r * 64 + lane, &key)) {
        const int id = hash_find(hk, hv, mask, key);
        if (id >= 0) {
          b = cstart[id];
          e = cstart[id + 1];
        }
      }
      const bool wide = e - b > kMsSerial;
      if (!wide) {
        for (int p0 = b; p0 < e; p0 += 4) {
          float4 x[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) x[k] = ptsS[min(p0 + k, e - 1)];
#pragma unroll
          for (int k = 0; k < 4; ++k) ms_take<D>(x[k], p0 + k < e, s, h2, acc, in);
        }
      }
      const uint64_t bm = __ballot(wide);
      if (wide) {
        const int pos = __popcll(bm & below);
        wb[r][pos] = b;
        we[r][pos] = e;
      }
      if (lane == 0) wn[r] = __popcll(bm);
    }
    __syncthreads();                                                  // 1
    for (int r = 0; r < NR; ++r) {
      const int nw = wn[r];
      for (int k = 0; k < nw; ++k) {
        const int bw = wb[r][k], ew = we[r][k];
        for (int p0 = bw + (int)threadIdx.x; p0 < ew; p0 += 4 * kMsThreads) {
          float4 x[4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) x[kk] = ptsS[min(p0 + kMsThreads * kk, ew - 1)];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
            ms_take<D>(x[kk], p0 + kMsThreads * kk < ew, s, h2, acc, in);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = wave_sum_f64(acc[j]);
    in = wave_sum_i32(in);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < D; ++j) part[w][j] = acc[j];
      part[w][D] = (double)in;
    }
    __syncthreads();                                                  // 2
    double tot[D];
#pragma unroll
    for (int j = 0; j < D; ++j) tot[j] = part[0][j];
    int tin = (int)part[0][D];
#pragma unroll
    for (int v = 1; v < NW; ++v) {
#pragma unroll
      for (int j = 0; j < D; ++j) tot[j] = tot[j] + part[v][j];
      tin += (int)part[v][D];
    }
    if (tin == 0) break;   // uniform: every thread read the same sums
    cnt = tin;
    double d[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double v = tot[j] / (double)tin;
      d[j] = v - s[j];
      s[j] = v;
    }
    if (sqrt(sq_norm<D>(d)) <= stop || it == max_iter) break;
    ++it;
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < D; ++j) mode[(size_t)c * D + j] = s[j];
    weight[c] = cnt;
    iters[c] = it;
    atomicMax(max_it, it);
  }
}

// ------------------------------------------------------------------ merge
// status: 0 undecided, 1 kept, 2 removed by a kept mode, 3 dropped seed.
__global__ __launch_bounds__(kSortThreads) void ms_status_init_kernel(
    const int *__restrict__ weight, const int *__restrict__ nsp, int *__restrict__ status) {
  const int i = blockIdx.x * kSortThreads + threadIdx.x;
  if (i < *nsp) status[i] = weight[i] > 0 ? 0 : 3;
}

// cnt[0] = carry, cnt[1 .. kRoundBatch] = 0 (carry: the undecided count of
// the previous batch's last round, or 1 before the first round).
__global__ void ms_round_clear_kernel(unsigned *__restrict__ cnt, int first) {
  const int t = threadIdx.x;
  const unsigned carry = first ? 1u : cnt[kRoundBatch];
  __syncthreads();
  if (t <= kRoundBatch) cnt[t] = (t == 0) ? carry : 0u;
}

// Does mode j come before mode i in the merge order?
template <int D>
__device__ __forceinline__ bool precedes(int j, int wj, const double *mj, int i, int wi,
                                         const double *mi) {
  if (wj != wi) return wj > wi;
#pragma unroll
  for (int k = 0; k < D; ++k)
    if (mj[k] != mi[k]) return mj[k] > mi[k];
  return j < i;
}

// One merge round, one wave per undecided mode: removed if a kept
// predecessor lies within h, kept if every predecessor within h is decided
// and none is kept, else counted in cnt[round].
template <int D>
__global__ __launch_bounds__(kMsThreads) void ms_merge_round_kernel(
    const double *__restrict__ mode, const int *__restrict__ weight,
    const int *__restrict__ nsp, const unsigned *__restrict__ perm2,
    const int *__restrict__ mstart, const uint64_t *__restrict__ hk,
    const int *__restrict__ hv, uint64_t mask, double h, int *status,
    unsigned *__restrict__ cnt, int round) {
  if (cnt[round - 1] == 0u) return;   // every mode decided already
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * kMsWaves + (threadIdx.x >> 6);
  if (i >= *nsp) return;
  volatile int *vst = status;
  if (vst[i] != 0) return;
  double mi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) mi[k] = mode[(size_t)i * D + k];
  const int wi = weight[i];
  const double h2 = h * h;
  GridQuery<D> g;
  g.init(mi, h);
  bool kept_pred = false, open_pred = false;
  for (int u0 = 0; u0 < (1 << (2 * D)); u0 += 64) {
    uint64_t key;
    if (!g.slot_key(u0 + lane, &key)) continue;
    const int id = hash_find(hk, hv, mask, key);
    if (id < 0) continue;
    const int p1 = mstart[id + 1];
    for (int p = mstart[id]; p < p1; ++p) {
      const int j = (int)perm2[p];
      if (j == i) continue;
      const int st = vst[j];
      if (st >= 2) continue;
      double mj[D], d[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        mj[k] = mode[(size_t)j * D + k];
        d[k] = mi[k] - mj[k];
      }
      if (sq_norm<D>(d) <= h2 && precedes<D>(j, weight[j], mj, i, wi, mi)) {
        if (st == 1) kept_pred = true;
        else open_pred = true;
      }
    }
  }
  const bool kept = __ballot(kept_pred) != 0ull;
  const bool open = __ballot(open_pred) != 0ull;
  if (lane == 0) {
    if (kept) vst[i] = 2;
    else if (!open) vst[i] = 1;
    else atomicAdd(&cnt[round], 1u);
  }
}

// The status word and the counters to the host's info block.
struct MsCounters {
  int ncells;    // seeds
  int nmodes;    // cells of the mode grid
  int kept;      // K
  int max_it;
  uint32_t status;
};

__global__ void ms_init_kernel(MsCounters *__restrict__ c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->ncells = 0;
    c->nmodes = 0;
    c->kept = 0;
    c->max_it = 0;
    c->status = 0u;
  }
}

}  // namespace gbms_dev
