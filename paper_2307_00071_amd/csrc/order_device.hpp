// Spatial ordering of the staged points (device code, included by gmm.hip).
//
// Tile culling skips (tile, component) pairs by a bound on the tile's
// bounding sphere, so it pays only when consecutive points are close in
// space.  Before a culled fit, the staged points are put in Morton
// (Z-order) order of a 256^3 grid over their bounding box:
//   bbox_kernel      per-block partial boxes (no atomics);
//   morton_kernel    every block reduces the partial boxes, then the 24-bit
//                    key of each point (padding gets the largest key);
//   radix passes     a stable LSD radix sort of (key, index), three 8-bit
//                    digits: per-block digit counts, a scan over the blocks
//                    of each digit (one block per digit), a stable scatter
//                    (digit starts from the digit totals; ranks from wave
//                    ballots, waves and rounds in item order);
//   gather_kernel    the points in sorted order.
// Every step is deterministic, so a fit is still bitwise reproducible, and
// no step clears memory with a memset (the fit may be captured in a graph).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "radix_device.hpp"

namespace gmm_dev {

constexpr int kBoxBlocks = 256;

__device__ inline void box_update(float4 x, float *lo, float *hi) {
  lo[0] = fminf(lo[0], x.x); lo[1] = fminf(lo[1], x.y); lo[2] = fminf(lo[2], x.z);
  hi[0] = fmaxf(hi[0], x.x); hi[1] = fmaxf(hi[1], x.y); hi[2] = fmaxf(hi[2], x.z);
}

// Min / max over a 256-thread block; thread 0 gets the result.
__device__ inline void box_block_reduce(float *lo, float *hi, float *sh /*4 x 6*/) {
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
    for (int v = 1; v < kSortThreads / 64; ++v)
      for (int j = 0; j < 3; ++j) {
        lo[j] = fminf(lo[j], sh[v * 6 + j]);
        hi[j] = fmaxf(hi[j], sh[v * 6 + 3 + j]);
      }
}

// Partial bounding boxes of the n real points: part6[block] = (lo, hi).
__global__ __launch_bounds__(kSortThreads) void bbox_kernel(
    const float4 *__restrict__ pts, int64_t n, float *__restrict__ part6) {
  __shared__ float sh[kSortThreads / 64 * 6];
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kSortThreads)
    box_update(pts[i], lo, hi);
  box_block_reduce(lo, hi, sh);
  if (threadIdx.x == 0)
    for (int j = 0; j < 3; ++j) {
      part6[blockIdx.x * 6 + j] = lo[j];
      part6[blockIdx.x * 6 + 3 + j] = hi[j];
    }
}

// 8 bits of v spread to every third bit.
__device__ inline unsigned spread3(unsigned v) {
  v &= 0xFFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// keys[i] = Morton code of point i in a cubic 256^3 grid over the box of
// the real points, 0xFFFFFF for padding; vals[i] = i.
__global__ __launch_bounds__(kSortThreads) void morton_kernel(
    const float4 *__restrict__ pts, int64_t n, int64_t npad,
    const float *__restrict__ part6, int nbox, unsigned *__restrict__ keys,
    unsigned *__restrict__ vals) {
  __shared__ float sh[kSortThreads / 64 * 6];
  __shared__ float box[4];
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nbox; b += kSortThreads) {
    for (int j = 0; j < 3; ++j) {
      lo[j] = fminf(lo[j], part6[b * 6 + j]);
      hi[j] = fmaxf(hi[j], part6[b * 6 + 3 + j]);
    }
  }
  box_block_reduce(lo, hi, sh);
  if (threadIdx.x == 0) {
    const float ext = fmaxf(fmaxf(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
    box[0] = lo[0];
    box[1] = lo[1];
    box[2] = lo[2];
    box[3] = (ext > 0.0f && ext < INFINITY) ? 255.99f / ext : 0.0f;
  }
  __syncthreads();
  const float l0 = box[0], l1 = box[1], l2 = box[2], sc = box[3];
  for (int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x; i < npad;
       i += (int64_t)gridDim.x * kSortThreads) {
    unsigned key = 0xFFFFFFu;
    if (i < n) {
      const float4 x = pts[i];
      const unsigned q0 = (unsigned)fminf(fmaxf((x.x - l0) * sc, 0.0f), 255.0f);
      const unsigned q1 = (unsigned)fminf(fmaxf((x.y - l1) * sc, 0.0f), 255.0f);
      const unsigned q2 = (unsigned)fminf(fmaxf((x.z - l2) * sc, 0.0f), 255.0f);
      key = spread3(q0) | (spread3(q1) << 1) | (spread3(q2) << 2);
    }
    keys[i] = key;
    vals[i] = (unsigned)i;
  }
}

// ---- batched fits: every frame in its own Morton order, frames kept in
// place.  Keys are (frame << 24) | Morton code in the frame's own box, so a
// four-pass sort of all staged points leaves each frame's range where it
// was (its padding, key (frame << 24) | 0xFFFFFF, at its end).
// (BFrame: the batched frame table of em_device.hpp, included first.)
// One block per frame: box6[f] = (lo, hi) of the frame's points.
__global__ __launch_bounds__(kSortThreads) void frame_box_kernel(
    const float4 *__restrict__ pts, const BFrame *__restrict__ frames, int tpts,
    float *__restrict__ box6) {
  __shared__ float sh[kSortThreads / 64 * 6];
  const BFrame F = frames[blockIdx.x];
  const float4 *p = pts + F.toff * tpts;
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = threadIdx.x; i < F.n; i += kSortThreads) box_update(p[i], lo, hi);
  box_block_reduce(lo, hi, sh);
  if (threadIdx.x == 0)
    for (int j = 0; j < 3; ++j) {
      box6[blockIdx.x * 6 + j] = lo[j];
      box6[blockIdx.x * 6 + 3 + j] = hi[j];
    }
}

// Keys of frame blockIdx.y over its staged range of fpad points (a
// multiple of the culled tile), starting at tile toff of tpts points.
__global__ __launch_bounds__(kSortThreads) void morton_frames_kernel(
    const float4 *__restrict__ pts, const BFrame *__restrict__ frames, int tpts,
    int pad_to, const float *__restrict__ box6, unsigned *__restrict__ keys,
    unsigned *__restrict__ vals) {
  const int f = blockIdx.y;
  const BFrame F = frames[f];
  const float l0 = box6[f * 6], l1 = box6[f * 6 + 1], l2 = box6[f * 6 + 2];
  const float ext = fmaxf(fmaxf(box6[f * 6 + 3] - l0, box6[f * 6 + 4] - l1),
                          box6[f * 6 + 5] - l2);
  const float sc = (ext > 0.0f && ext < INFINITY) ? 255.99f / ext : 0.0f;
  const long long s0 = F.toff * tpts;
  const int n = F.n, np = ((n + pad_to - 1) / pad_to) * pad_to;
  for (int i = blockIdx.x * kSortThreads + threadIdx.x; i < np;
       i += gridDim.x * kSortThreads) {
    unsigned key = 0xFFFFFFu;
    if (i < n) {
      const float4 x = pts[s0 + i];
      const unsigned q0 = (unsigned)fminf(fmaxf((x.x - l0) * sc, 0.0f), 255.0f);
      const unsigned q1 = (unsigned)fminf(fmaxf((x.y - l1) * sc, 0.0f), 255.0f);
      const unsigned q2 = (unsigned)fminf(fmaxf((x.z - l2) * sc, 0.0f), 255.0f);
      key = spread3(q0) | (spread3(q1) << 1) | (spread3(q2) << 2);
    }
    keys[s0 + i] = ((unsigned)f << 24) | key;
    vals[s0 + i] = (unsigned)(s0 + i);
  }
}

// out[i] = in[perm[i]]
__global__ __launch_bounds__(kSortThreads) void gather_kernel(
    const float4 *__restrict__ in, const unsigned *__restrict__ perm,
    int64_t npad, float4 *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kSortThreads + threadIdx.x;
  if (i < npad) out[i] = in[perm[i]];
}

}  // namespace gmm_dev
