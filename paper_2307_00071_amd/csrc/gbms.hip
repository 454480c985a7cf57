// MI355X (gfx950) mean shift for the number of mixture components: host side
// of the C ABI call gmm_meanshift (include/gmm.h).  Kernels in
// gbms_device.hpp.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "gbms_device.hpp"
#include "gmm.h"

namespace gmm_host {
extern thread_local char g_err[512];
}

namespace {

using namespace gbms_dev;
using gmm_host::g_err;

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

template <typename T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<unsigned char *>(ws) + off);
}

unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Workspace of a call with n points in D dimensions (every buffer 256-byte
// aligned).  The point grid's buffers are reused for the mode grid once the
// seeds have converged.
struct MsLayout {
  int64_t n = 0;
  int nblk = 0;           // radix / scan blocks
  uint64_t cap = 0;       // hash slots (a power of two >= 2 n)
  size_t cnt, rounds;     // MsCounters; kRoundBatch + 1 round counters
  size_t klo, khi, vals;  // keys of the items, identity values
  size_t kA, vA, kB, vB;  // radix ping-pong
  size_t hist, dtot;
  size_t keys;            // sorted 64-bit keys
  size_t ptsS;            // sorted points (float4)
  size_t start;           // cell starts, n + 1
  size_t ckey;            // cell keys
  size_t hk, hv;          // hash table
  size_t mode, weight, iters, status;
  size_t total;
};

MsLayout ms_layout(int64_t n, int d) {
  MsLayout L;
  L.n = n;
  L.nblk = (int)std::max<int64_t>(1, (n + kSortChunk - 1) / kSortChunk);
  L.cap = 256;
  while (L.cap < 2 * (uint64_t)n) L.cap <<= 1;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at_ = o;
    o = align256(o + bytes);
    return at_;
  };
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  L.cnt = take(sizeof(MsCounters));
  L.rounds = take((kRoundBatch + 1) * sizeof(unsigned));
  L.klo = take(nn * 4);
  L.khi = take(nn * 4);
  L.vals = take(nn * 4);
  L.kA = take(nn * 4);
  L.vA = take(nn * 4);
  L.kB = take(nn * 4);
  L.vB = take(nn * 4);
  L.hist = take((size_t)256 * L.nblk * 4);
  L.dtot = take(256 * 4);
  L.keys = take(nn * 8);
  L.ptsS = take(nn * 16);
  L.start = take((nn + 1) * 4);
  L.ckey = take(nn * 8);
  L.hk = take(L.cap * 8);
  L.hv = take(L.cap * 4);
  L.mode = take(nn * d * 8);
  L.weight = take(nn * 4);
  L.iters = take(nn * 4);
  L.status = take(nn * 4);
  L.total = o;
  return L;
}

struct WsGuard {
  void *ptr = nullptr;
  hipStream_t s = nullptr;
  ~WsGuard() {
    if (ptr) (void)hipFreeAsync(ptr, s);
  }
};

// Stable sort of the n (khi:klo) keys: four 8-bit passes over the low
// words (values = identity), the high words gathered through the values,
// four passes over them.  The permutation ends in vA.
gmm_status sort64(const MsLayout &L, void *ws, hipStream_t s, int64_t n) {
  using namespace gmm_dev;
  const int nblk = L.nblk;
  unsigned *hist = at<unsigned>(ws, L.hist), *dtot = at<unsigned>(ws, L.dtot);
  auto pass = [&](const unsigned *kin, const unsigned *vin, int shift, unsigned *kout,
                  unsigned *vout) -> gmm_status {
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nblk), dim3(kSortThreads), 0, s, kin, n,
                       shift, hist, nblk);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(radix_scan_kernel, dim3(256), dim3(kSortThreads), 0, s, hist, nblk,
                       dtot);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblk), dim3(kSortThreads), 0, s, kin, vin,
                       n, shift, hist, nblk, dtot, kout, vout);
    HIP_TRY(hipGetLastError());
    return GMM_OK;
  };
  unsigned *kA = at<unsigned>(ws, L.kA), *vA = at<unsigned>(ws, L.vA);
  unsigned *kB = at<unsigned>(ws, L.kB), *vB = at<unsigned>(ws, L.vB);
  gmm_status st;
  if ((st = pass(at<unsigned>(ws, L.klo), at<unsigned>(ws, L.vals), 0, kB, vB)) != GMM_OK) return st;
  if ((st = pass(kB, vB, 8, kA, vA)) != GMM_OK) return st;
  if ((st = pass(kA, vA, 16, kB, vB)) != GMM_OK) return st;
  if ((st = pass(kB, vB, 24, kA, vA)) != GMM_OK) return st;
  hipLaunchKernelGGL(ms_gather_u32_kernel, dim3(blocks(n, kSortThreads)), dim3(kSortThreads), 0,
                     s, at<unsigned>(ws, L.khi), vA, (const int *)nullptr, n, kA);
  HIP_TRY(hipGetLastError());
  if ((st = pass(kA, vA, 0, kB, vB)) != GMM_OK) return st;
  if ((st = pass(kB, vB, 8, kA, vA)) != GMM_OK) return st;
  if ((st = pass(kA, vA, 16, kB, vB)) != GMM_OK) return st;
  if ((st = pass(kB, vB, 24, kA, vA)) != GMM_OK) return st;
  return GMM_OK;
}

// Cells of the n sorted keys: start (n + 1), ckey, the count to *ncount;
// then the hash table of the cells.
gmm_status build_grid(const MsLayout &L, void *ws, hipStream_t s, int64_t n, int *ncount) {
  using namespace gmm_dev;
  const int nblk = L.nblk;
  unsigned *bsum = at<unsigned>(ws, L.hist), *dtot = at<unsigned>(ws, L.dtot);
  const uint64_t *keys = at<uint64_t>(ws, L.keys);
  hipLaunchKernelGGL(ms_flag_count_kernel<FLAG_CELL>, dim3(nblk), dim3(kSortThreads), 0, s,
                     keys, (const int *)nullptr, (const int *)nullptr, n, bsum);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(radix_scan_kernel, dim3(1), dim3(kSortThreads), 0, s, bsum, nblk, dtot);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL((ms_flag_write_kernel<FLAG_CELL, 3>), dim3(nblk), dim3(kSortThreads), 0, s,
                     keys, (const int *)nullptr, (const int *)nullptr, n, bsum,
                     at<int>(ws, L.start), at<uint64_t>(ws, L.ckey), (const double *)nullptr,
                     (const int *)nullptr, (double *)nullptr, (long long *)nullptr, (int64_t)0);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(ms_cells_end_kernel, dim3(1), dim3(64), 0, s, dtot, (const int *)nullptr, n,
                     at<int>(ws, L.start), ncount);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(ms_hash_clear_kernel, dim3(blocks((int64_t)L.cap, kSortThreads)),
                     dim3(kSortThreads), 0, s, at<uint64_t>(ws, L.hk), L.cap);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(ms_hash_insert_kernel, dim3(blocks(n, kSortThreads)), dim3(kSortThreads), 0,
                     s, at<uint64_t>(ws, L.ckey), ncount, at<uint64_t>(ws, L.hk),
                     at<int>(ws, L.hv), L.cap - 1);
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

template <int D>
gmm_status run_meanshift(const MsLayout &L, void *ws, hipStream_t s, const float *pts,
                         int64_t n, double h, int max_iter, double *modes, int64_t *weights,
                         int64_t max_modes, double *seed_mode, int *seed_w, int *seed_it,
                         int *seed_st, gmm_meanshift_info *info) {
  MsCounters *cnt = at<MsCounters>(ws, L.cnt);
  unsigned *rc = at<unsigned>(ws, L.rounds);
  double *mode = seed_mode ? seed_mode : at<double>(ws, L.mode);
  int *weight = seed_w ? seed_w : at<int>(ws, L.weight);
  int *iters = seed_it ? seed_it : at<int>(ws, L.iters);
  int *status = seed_st ? seed_st : at<int>(ws, L.status);
  hipLaunchKernelGGL(ms_init_kernel, dim3(1), dim3(64), 0, s, cnt);
  HIP_TRY(hipGetLastError());

  // ---- the point grid: keys, sort, cells (= seeds), hash table
  hipLaunchKernelGGL(ms_point_key_kernel<D>, dim3(blocks(n, kSortThreads)), dim3(kSortThreads),
                     0, s, pts, n, h, at<unsigned>(ws, L.klo), at<unsigned>(ws, L.khi),
                     at<unsigned>(ws, L.vals), &cnt->status);
  HIP_TRY(hipGetLastError());
  gmm_status st;
  if ((st = sort64(L, ws, s, n)) != GMM_OK) return st;
  hipLaunchKernelGGL(ms_sorted_kernel<D>, dim3(blocks(n, kSortThreads)), dim3(kSortThreads), 0,
                     s, at<unsigned>(ws, L.klo), at<unsigned>(ws, L.khi),
                     at<unsigned>(ws, L.vA), pts, (const int *)nullptr, n,
                     at<uint64_t>(ws, L.keys), at<float4>(ws, L.ptsS));
  HIP_TRY(hipGetLastError());
  if ((st = build_grid(L, ws, s, n, &cnt->ncells)) != GMM_OK) return st;

  // ---- every seed to its mode (at most n seeds; the count is on the
  // device): one wave per seed, or a block per seed when there are at most
  // thr seeds; each kernel returns at once when the other one applies.
  // GMM_MS_SEED_WAVES=1|4 forces one form (tests of both on one input).
  int thr = kMsBlockSeeds;
  if (const char *e = getenv("GMM_MS_SEED_WAVES")) {
    if (e[0] == '1') thr = 0;
    if (e[0] == '4') thr = (int)std::min<int64_t>(n, INT32_MAX);
  }
  hipLaunchKernelGGL(ms_shift_kernel<D>, dim3(blocks(n, kMsWaves)), dim3(kMsThreads), 0, s,
                     at<float4>(ws, L.ptsS), at<int>(ws, L.start), at<uint64_t>(ws, L.ckey),
                     &cnt->ncells, at<uint64_t>(ws, L.hk), at<int>(ws, L.hv), L.cap - 1, h,
                     max_iter, mode, weight, iters, &cnt->max_it, thr);
  HIP_TRY(hipGetLastError());
  if (thr > 0) {
    hipLaunchKernelGGL(ms_shift4_kernel<D>, dim3((unsigned)std::min<int64_t>(n, thr)),
                       dim3(kMsThreads), 0, s, at<float4>(ws, L.ptsS), at<int>(ws, L.start),
                       at<uint64_t>(ws, L.ckey), &cnt->ncells, at<uint64_t>(ws, L.hk),
                       at<int>(ws, L.hv), L.cap - 1, h, max_iter, mode, weight, iters,
                       &cnt->max_it, thr);
    HIP_TRY(hipGetLastError());
  }

  // ---- the mode grid over the same buffers; perm2 (sorted -> seed) in vA
  hipLaunchKernelGGL(ms_mode_key_kernel<D>, dim3(blocks(n, kSortThreads)), dim3(kSortThreads),
                     0, s, mode, weight, &cnt->ncells, n, h, at<unsigned>(ws, L.klo),
                     at<unsigned>(ws, L.khi), at<unsigned>(ws, L.vals));
  HIP_TRY(hipGetLastError());
  if ((st = sort64(L, ws, s, n)) != GMM_OK) return st;
  hipLaunchKernelGGL(ms_sorted_kernel<D>, dim3(blocks(n, kSortThreads)), dim3(kSortThreads), 0,
                     s, at<unsigned>(ws, L.klo), at<unsigned>(ws, L.khi),
                     at<unsigned>(ws, L.vA), (const float *)nullptr, (const int *)nullptr, n,
                     at<uint64_t>(ws, L.keys), (float4 *)nullptr);
  HIP_TRY(hipGetLastError());
  if ((st = build_grid(L, ws, s, n, &cnt->nmodes)) != GMM_OK) return st;

  // ---- merge rounds, kRoundBatch launches per check of the last count
  hipLaunchKernelGGL(ms_status_init_kernel, dim3(blocks(n, kSortThreads)), dim3(kSortThreads), 0,
                     s, weight, &cnt->ncells, status);
  HIP_TRY(hipGetLastError());
  int rounds = 0;
  for (int batch = 0;; ++batch) {
    hipLaunchKernelGGL(ms_round_clear_kernel, dim3(1), dim3(64), 0, s, rc, batch == 0 ? 1 : 0);
    HIP_TRY(hipGetLastError());
    for (int r = 1; r <= kRoundBatch; ++r) {
      hipLaunchKernelGGL(ms_merge_round_kernel<D>, dim3(blocks(n, kMsWaves)), dim3(kMsThreads), 0,
                         s, mode, weight, &cnt->ncells, at<unsigned>(ws, L.vA),
                         at<int>(ws, L.start), at<uint64_t>(ws, L.hk), at<int>(ws, L.hv),
                         L.cap - 1, h, status, rc, r);
      HIP_TRY(hipGetLastError());
    }
    unsigned hc[kRoundBatch + 1];
    HIP_TRY(hipMemcpyAsync(hc, rc, sizeof hc, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int r = 1;
    while (r <= kRoundBatch && hc[r] != 0u) ++r;
    if (r <= kRoundBatch) {
      rounds += r;
      break;
    }
    rounds += kRoundBatch;
    if (rounds > n + kRoundBatch)   // each round decides a mode: cannot happen
      return fail(GMM_ERR_DEVICE, "merge did not finish after %d rounds", rounds);
  }

  // ---- the kept modes in seed order
  {
    using namespace gmm_dev;
    const int nblk = L.nblk;
    unsigned *bsum = at<unsigned>(ws, L.hist), *dtot = at<unsigned>(ws, L.dtot);
    hipLaunchKernelGGL(ms_flag_count_kernel<FLAG_KEPT>, dim3(nblk), dim3(kSortThreads), 0, s,
                       (const uint64_t *)nullptr, status, &cnt->ncells, n, bsum);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(radix_scan_kernel, dim3(1), dim3(kSortThreads), 0, s, bsum, nblk, dtot);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL((ms_flag_write_kernel<FLAG_KEPT, D>), dim3(nblk), dim3(kSortThreads), 0, s,
                       (const uint64_t *)nullptr, status, &cnt->ncells, n, bsum, (int *)nullptr,
                       (uint64_t *)nullptr, mode, weight, modes,
                       reinterpret_cast<long long *>(weights), max_modes);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(ms_cells_end_kernel, dim3(1), dim3(64), 0, s, dtot,
                       (const int *)nullptr, (int64_t)0, at<int>(ws, L.start), &cnt->kept);
    HIP_TRY(hipGetLastError());
  }
  MsCounters hcnt;
  HIP_TRY(hipMemcpyAsync(&hcnt, cnt, sizeof hcnt, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  info->n_seeds = hcnt.ncells;
  info->n_modes = hcnt.kept;
  info->rounds = rounds;
  info->max_iters = hcnt.max_it;
  if (hcnt.status & kMsNonFinite) return fail(GMM_ERR_NONFINITE, "non-finite point coordinate");
  if (hcnt.status & kMsRange)
    return fail(GMM_ERR_INVALID_ARG,
                "a bin index |x / h| exceeds %lld: bandwidth too small for the cloud's extent",
                (long long)((1ll << (KeyBits<D>::v - 1)) - 2));
  if (hcnt.kept > max_modes)
    return fail(GMM_ERR_INVALID_ARG, "%d modes kept, the output holds %lld", hcnt.kept,
                (long long)max_modes);
  return GMM_OK;
}

}  // namespace

extern "C" {

size_t gmm_meanshift_workspace_size(int64_t n, int32_t d) {
  if (n < 0 || (d != 3 && d != 4)) return 0;
  return ms_layout(n, d).total;
}

gmm_status gmm_meanshift(const float *pts, int64_t n, int32_t d, double bandwidth,
                         int32_t max_iter, double *modes, int64_t *weights, int64_t max_modes,
                         double *seed_modes, int32_t *seed_weights, int32_t *seed_iters,
                         int32_t *seed_status, gmm_meanshift_info *info, void *ws,
                         size_t ws_bytes, void *stream) {
  if (!info) return fail(GMM_ERR_INVALID_ARG, "info must not be NULL");
  memset(info, 0, sizeof *info);
  if (d != 3 && d != 4) return fail(GMM_ERR_INVALID_ARG, "d must be 3 or 4, got %d", d);
  if (n < 0 || n > (int64_t)INT32_MAX - 1)
    return fail(GMM_ERR_INVALID_ARG, "n must be in [0, 2^31 - 1), got %lld", (long long)n);
  if (!(bandwidth > 0.0) || !isfinite(bandwidth))
    return fail(GMM_ERR_INVALID_ARG, "bandwidth must be finite and > 0");
  if (max_iter < 0) return fail(GMM_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (max_modes < 0) return fail(GMM_ERR_INVALID_ARG, "max_modes must be >= 0");
  if (n == 0) return GMM_OK;
  if (!pts || (max_modes > 0 && !modes))
    return fail(GMM_ERR_INVALID_ARG, "pts and modes must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const MsLayout L = ms_layout(n, d);
  WsGuard guard;
  if (ws == nullptr) {
    const char *fi = getenv("GMM_FAULT_INJECT");
    if (fi && strcmp(fi, "oom") == 0)
      return fail(GMM_ERR_OOM, "hipMallocAsync(%zu) failed (GMM_FAULT_INJECT=oom)", L.total);
    if (hipMallocAsync(&ws, L.total, s) != hipSuccess)
      return fail(GMM_ERR_OOM, "hipMallocAsync(%zu) failed", L.total);
    guard.ptr = ws;
    guard.s = s;
    ws_bytes = L.total;
  }
  if (ws_bytes < L.total)
    return fail(GMM_ERR_OOM, "workspace %zu bytes < %zu needed", ws_bytes, L.total);
  if (reinterpret_cast<uintptr_t>(ws) & 255)
    return fail(GMM_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (d == 3)
    return run_meanshift<3>(L, ws, s, pts, n, bandwidth, max_iter, modes, weights, max_modes,
                            seed_modes, seed_weights, seed_iters, seed_status, info);
  return run_meanshift<4>(L, ws, s, pts, n, bandwidth, max_iter, modes, weights, max_modes,
                          seed_modes, seed_weights, seed_iters, seed_status, info);
}

}  // extern "C"
