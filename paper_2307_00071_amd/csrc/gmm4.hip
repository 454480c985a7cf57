// MI355X (gfx950) 4D mixture (x, y, z, intensity): host side of the C ABI
// calls gmm4_fit, gmm4_color_conditional and gmm4_joint_dist_sample
// (include/gmm.h).  Kernels in em4_device.hpp.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "em4_device.hpp"
#include "gmm.h"
#include "radix_device.hpp"

namespace gmm_host {
extern thread_local char g_err[512];
}

namespace {

using namespace gmm4_dev;
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

int device_cus() {
  static std::mutex mu;
  static int cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  std::lock_guard<std::mutex> lk(mu);
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      cache[dev] = v;
  }
  return cache[dev];
}

gmm_status status_from_bits(uint32_t bits) {
  if (bits & kStBadArg) return fail(GMM_ERR_INVALID_ARG, "device: invalid label or parameter");
  if (bits & kStNotSpd) return fail(GMM_ERR_NOT_SPD, "device: covariance not SPD");
  if (bits & kStNonFinite) return fail(GMM_ERR_NONFINITE, "device: non-finite value");
  return GMM_OK;
}

struct WsGuard {
  void *ptr = nullptr;
  hipStream_t s = nullptr;
  ~WsGuard() {
    if (ptr) (void)hipFreeAsync(ptr, s);
  }
};

gmm_status get_ws(void **ws, size_t *ws_bytes, size_t need, hipStream_t s, WsGuard *g) {
  if (*ws == nullptr) {
    void *p = nullptr;
    // GMM_FAULT_INJECT=oom: the allocation fails (tests of the error path)
    const char *fi = getenv("GMM_FAULT_INJECT");
    if (fi && strcmp(fi, "oom") == 0)
      return fail(GMM_ERR_OOM, "hipMallocAsync(%zu) failed (GMM_FAULT_INJECT=oom)", need);
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

// ----------------------------------------------------------------- fit
struct Cfg4 {
  int P = 0, trip = 0, grid = 0;
  size_t lds = 0;
  const void *kfn = nullptr;
  void (*launch)(const Cfg4 &, hipStream_t, const float4 *, const int32_t *, const float *,
                 const float4 *, double *, const Tile4Args &) = nullptr;
};

template <int TRIP>
void launch_tile4(const Cfg4 &c, hipStream_t s, const float4 *pts, const int32_t *lab,
                  const float *cpar, const float4 *shift, double *part, const Tile4Args &a) {
  hipLaunchKernelGGL(em4_tile_kernel<TRIP>, dim3(c.grid), dim3(kBlock), c.lds, s, pts, lab,
                     cpar, shift, part, a);
}

// Point subsets per component: the largest power of two P with P K <= the
// block and P <= kT; TRIP = kT / P points each.
bool make_cfg4(int K, int64_t n, Cfg4 *c) {
  const int cus = device_cus();
  if (cus <= 0 || K < 1 || K > kMaxK) return false;
  int P = 1;
  while (P * 2 <= kT && P * 2 * K <= kBlock) P *= 2;
  c->P = P;
  c->trip = kT / P;
  switch (c->trip) {
#define GMM4_TRIP(TR)                                                       \
  case TR:                                                                  \
    c->launch = &launch_tile4<TR>;                                          \
    c->kfn = reinterpret_cast<const void *>(&em4_tile_kernel<TR>);          \
    break;
    GMM4_TRIP(1) GMM4_TRIP(2) GMM4_TRIP(4) GMM4_TRIP(8) GMM4_TRIP(16) GMM4_TRIP(32)
    GMM4_TRIP(64)
#undef GMM4_TRIP
    default: return false;
  }
  c->lds = tile4_lds_bytes(K);
  if (c->lds > 65536 && hipFuncSetAttribute(c->kfn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)c->lds) != hipSuccess)
    return false;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c->kfn, kBlock, c->lds) !=
          hipSuccess || per_cu <= 0)
    return false;
  const int64_t ntiles = (n + kT - 1) / kT;
  c->grid = (int)std::max<int64_t>(1, std::min<int64_t>(ntiles, (int64_t)cus * per_cu));
  return true;
}

// Culled soft passes (em4_cull_kernel) over the points in Morton order of
// their xyz part; GMM_CULL4=0 keeps the dense kernel for every pass.
struct CullCfg4 {
  bool on = false;
  int grid = 0, scap = 0, nw = 0;
  size_t lds = 0;
  const void *kfn = nullptr;
};

bool cull4_enabled() {
  const char *e = getenv("GMM_CULL4");
  return !(e && e[0] == '0');
}

bool make_cull4(int K, int64_t n, CullCfg4 *c) {
  const int cus = device_cus();
  if (cus <= 0 || K < 1 || K > kMaxK) return false;
  // E rows: 128, or 256 above K = 256, where the FP64 sums leave LDS for
  // one block per CU either way
  c->scap = std::min(K, K > 256 ? 2 * kCull4Cap : kCull4Cap);
  c->nw = kCull4Waves;
  c->lds = cull4_lds(K, c->scap, c->nw).total;
  c->kfn = reinterpret_cast<const void *>(&em4_cull_kernel<kCull4Waves>);
  if (c->lds > 65536 &&
      hipFuncSetAttribute(c->kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds) !=
          hipSuccess)
    return false;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c->kfn, c->nw * 64, c->lds) !=
          hipSuccess || per_cu <= 0)
    return false;
  const int64_t ntiles = (n + kT - 1) / kT;
  c->grid = (int)std::max<int64_t>(1, std::min<int64_t>(ntiles, (int64_t)cus * per_cu));
  // GMM_CULL4_GRID=<blocks>: fewer persistent blocks (tuning experiments)
  if (const char *g = getenv("GMM_CULL4_GRID")) {
    const int v = atoi(g);
    if (v > 0 && v < c->grid) c->grid = v;
  }
  c->on = true;
  return true;
}

struct Layout4 {
  size_t status, cpar[2], shift[2], th64, red, part, total;
  int ncols;
  // culled passes: ordered points and labels, tile spheres, sort buffers
  size_t spts = 0, slab = 0, tsph = 0, keys[2] = {0, 0}, vals[2] = {0, 0}, hist = 0,
         dtot = 0, box6 = 0;
  int64_t npad = 0;
  int nblk = 0;
};

Layout4 layout4(int K, int grid, int64_t n = 0, bool cull = false) {
  Layout4 L{};
  size_t o = 0;
  L.ncols = kNStat * K + 1;
  L.status = o; o = align256(o + 256);
  for (int i = 0; i < 2; ++i) {
    L.cpar[i] = o; o = align256(o + (size_t)(K + 1) * kPar * sizeof(float));
    L.shift[i] = o; o = align256(o + (size_t)K * sizeof(float4));
  }
  L.th64 = o; o = align256(o + (size_t)K * kTh * sizeof(double));
  L.red = o; o = align256(o + (size_t)kRedChunks * L.ncols * sizeof(double));
  L.part = o; o = align256(o + (size_t)grid * L.ncols * sizeof(double));
  if (cull) {
    L.npad = ((n + kT - 1) / kT) * kT;
    L.nblk = (int)((L.npad + gmm_dev::kSortChunk - 1) / gmm_dev::kSortChunk);
    L.spts = o; o = align256(o + (size_t)L.npad * sizeof(float4));
    L.slab = o; o = align256(o + (size_t)L.npad * sizeof(int32_t));
    L.tsph = o; o = align256(o + (size_t)(L.npad / kT) * sizeof(float4));
    for (int i = 0; i < 2; ++i) {
      L.keys[i] = o; o = align256(o + (size_t)L.npad * sizeof(unsigned));
      L.vals[i] = o; o = align256(o + (size_t)L.npad * sizeof(unsigned));
    }
    L.hist = o; o = align256(o + (size_t)256 * L.nblk * sizeof(unsigned));
    L.dtot = o; o = align256(o + 256 * sizeof(unsigned));
    L.box6 = o; o = align256(o + (size_t)kBox4Blocks * 6 * sizeof(float));
  }
  L.total = o;
  return L;
}

struct Run4 {
  Cfg4 c;
  CullCfg4 cc;
  Layout4 L;
  void *ws = nullptr;
  hipStream_t s = nullptr;
  int K = 0, cur = 0;
  int64_t n = 0;
  const float4 *pts = nullptr;
  const int32_t *labels = nullptr;
  bool fused = false;   // lambda > 0: one reduction + update launch per pass
};

gmm_status pass4(Run4 &r, int mode, int umode, double reg, double *slot,
                 float *ow = nullptr, float *omu = nullptr, float *ocov = nullptr) {
  const Layout4 &L = r.L;
  Tile4Args a;
  a.n = r.n;
  a.ntiles = (int)((r.n + kT - 1) / kT);
  a.K = r.K;
  a.P = r.c.P;
  a.mode = mode;
  a.ncols = L.ncols;
  const bool fuse = r.fused && reg > 0.0;
  a.cmaj = fuse ? 1 : 0;
  const bool culled = r.cc.on && mode != kLabels;
  const int nrows = culled ? r.cc.grid : r.c.grid;
  if (culled) {
    Cull4Args ca;
    ca.n = r.n;
    ca.ntiles = a.ntiles;
    ca.K = r.K;
    ca.mode = mode;
    ca.ncols = L.ncols;
    ca.scap = r.cc.scap;
    ca.cmaj = a.cmaj;
    hipLaunchKernelGGL(em4_cull_kernel<kCull4Waves>, dim3(r.cc.grid), dim3(kCull4Waves * 64),
                       r.cc.lds, r.s, r.pts, at<float4>(r.ws, L.tsph),
                       at<float>(r.ws, L.cpar[r.cur]), at<float4>(r.ws, L.shift[r.cur]),
                       at<double>(r.ws, L.part), ca);
  } else {
    r.c.launch(r.c, r.s, r.pts, r.labels, at<float>(r.ws, L.cpar[r.cur]),
               at<float4>(r.ws, L.shift[r.cur]), at<double>(r.ws, L.part), a);
  }
  HIP_TRY(hipGetLastError());
  if (fuse) {
    const int nxt = 1 - r.cur;
    Fuse4Args fa;
    fa.K = r.K;
    fa.ncols = L.ncols;
    fa.nrows = nrows;
    fa.mode = mode;
    fa.umode = umode;
    fa.reg = reg;
    fa.Ntot = (double)r.n + r.K * kEpsN;
    fa.lnZ = log(fa.Ntot) - 2.0 * log(reg) - log((double)r.K);
    fa.Chdr = (-2.0 * log(reg) - 2.0 * kLn2Pi - log((double)r.K)) * kLog2e;
    hipLaunchKernelGGL(reduce_update4_kernel, dim3(r.K), dim3(kFuse4Threads), 0, r.s,
                       at<double>(r.ws, L.part), at<float>(r.ws, L.cpar[r.cur]),
                       at<float4>(r.ws, L.shift[r.cur]), at<float>(r.ws, L.cpar[nxt]),
                       at<float4>(r.ws, L.shift[nxt]), at<double>(r.ws, L.th64), slot, ow, omu,
                       ocov, at<uint32_t>(r.ws, L.status), fa);
    HIP_TRY(hipGetLastError());
    if (umode != kUpdNone) r.cur = nxt;
    return GMM_OK;
  }
  hipLaunchKernelGGL(reduce4_kernel, dim3((L.ncols + 255) / 256, kRedChunks), dim3(256), 0,
                     r.s, at<double>(r.ws, L.part), nrows, L.ncols, at<double>(r.ws, L.red));
  HIP_TRY(hipGetLastError());
  const int nxt = 1 - r.cur;
  Upd4Args ua;
  ua.K = r.K;
  ua.ncols = L.ncols;
  ua.mode = mode;
  ua.umode = umode;
  ua.chunks = kRedChunks;
  ua.reg = reg;
  hipLaunchKernelGGL(update4_kernel, dim3(1), dim3(kUpdThreads), 0, r.s,
                     at<double>(r.ws, L.red), at<float>(r.ws, L.cpar[r.cur]),
                     at<float4>(r.ws, L.shift[r.cur]), at<float>(r.ws, L.cpar[nxt]),
                     at<float4>(r.ws, L.shift[nxt]), at<double>(r.ws, L.th64), slot, ow, omu,
                     ocov, at<uint32_t>(r.ws, L.status), ua);
  HIP_TRY(hipGetLastError());
  if (umode != kUpdNone) r.cur = nxt;
  return GMM_OK;
}

gmm_status check_fit4(int64_t n, int32_t k) {
  if (n <= 0 || n > GMM_MAX_N) return fail(GMM_ERR_INVALID_ARG, "n=%lld out of range", (long long)n);
  if (k <= 0) return fail(GMM_ERR_INVALID_ARG, "k=%d must be positive", k);
  if (k > kMaxK) return fail(GMM_ERR_UNSUPPORTED, "k=%d above the 4D limit %d", k, kMaxK);
  if (k > n) return fail(GMM_ERR_INVALID_ARG, "k=%d > n=%lld", k, (long long)n);
  return GMM_OK;
}


// Culled fits: the points (and labels) in Morton order of their xyz part,
// and the bounding sphere of every 64-point tile; r.pts / r.labels then
// point at the ordered copies.  The sums of a pass are order-free, so only
// the order of floating-point additions changes.
gmm_status order4(Run4 &r) {
  const Layout4 &L = r.L;
  const int64_t n = r.n, npad = L.npad;
  hipLaunchKernelGGL(bbox4_kernel, dim3(kBox4Blocks), dim3(kOrd), 0, r.s, r.pts, n,
                     at<float>(r.ws, L.box6));
  HIP_TRY(hipGetLastError());
  const unsigned mb = (unsigned)std::min<int64_t>(256, (npad + kOrd - 1) / kOrd);
  hipLaunchKernelGGL(morton4_kernel, dim3(mb), dim3(kOrd), 0, r.s, r.pts, n, npad,
                     at<float>(r.ws, L.box6), kBox4Blocks, at<unsigned>(r.ws, L.keys[0]),
                     at<unsigned>(r.ws, L.vals[0]));
  HIP_TRY(hipGetLastError());
  int src = 0;
  for (int shift = 0; shift < 24; shift += 8, src = 1 - src) {
    hipLaunchKernelGGL(gmm_dev::radix_hist_kernel, dim3(L.nblk), dim3(gmm_dev::kSortThreads), 0,
                       r.s, at<unsigned>(r.ws, L.keys[src]), npad, shift,
                       at<unsigned>(r.ws, L.hist), L.nblk);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(gmm_dev::radix_scan_kernel, dim3(256), dim3(gmm_dev::kSortThreads), 0,
                       r.s, at<unsigned>(r.ws, L.hist), L.nblk, at<unsigned>(r.ws, L.dtot));
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(gmm_dev::radix_scatter_kernel, dim3(L.nblk), dim3(gmm_dev::kSortThreads),
                       0, r.s, at<unsigned>(r.ws, L.keys[src]), at<unsigned>(r.ws, L.vals[src]),
                       npad, shift, at<unsigned>(r.ws, L.hist), L.nblk,
                       at<unsigned>(r.ws, L.dtot), at<unsigned>(r.ws, L.keys[1 - src]),
                       at<unsigned>(r.ws, L.vals[1 - src]));
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(gather4_kernel, dim3((unsigned)((npad + kOrd - 1) / kOrd)), dim3(kOrd), 0,
                     r.s, r.pts, r.labels, at<unsigned>(r.ws, L.vals[src]), n, npad,
                     at<float4>(r.ws, L.spts), r.labels ? at<int32_t>(r.ws, L.slab) : nullptr);
  HIP_TRY(hipGetLastError());
  const int ntiles = (int)(npad / kT);
  hipLaunchKernelGGL(tile_sphere4_kernel, dim3((unsigned)((ntiles + kOrd / 64 - 1) / (kOrd / 64))),
                     dim3(kOrd), 0, r.s, at<float4>(r.ws, L.spts), n, ntiles,
                     at<float4>(r.ws, L.tsph));
  HIP_TRY(hipGetLastError());
  r.pts = at<float4>(r.ws, L.spts);
  if (r.labels) r.labels = at<int32_t>(r.ws, L.slab);
  return GMM_OK;
}

// The whole fit on r.s: init, checks, theta_0, T iterations, the final
// log-likelihood pass and the outputs.
gmm_status enqueue4(Run4 &r, float *w, float *mu, float *cov, double *loglik,
                    const gmm_fit_opts *opts) {
  const int k = r.K;
  const int64_t n = r.n;
  void *ws = r.ws;
  gmm_status st;
  hipLaunchKernelGGL(init4_kernel, dim3(1), dim3(256), 0, r.s, at<uint32_t>(ws, r.L.status),
                     r.labels ? at<float4>(ws, r.L.shift[0]) : nullptr, k);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(check4_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, r.s,
                     r.pts, r.labels, n, k, at<uint32_t>(ws, r.L.status));
  HIP_TRY(hipGetLastError());
  if (r.cc.on && (st = order4(r)) != GMM_OK) return st;
  const double reg = opts->reg_covar;
  r.cur = 0;
  if (r.labels) {
    // theta_0 = M-step of the one-hot responsibilities: the mean (shift 0),
    // then the scatter about it
    if ((st = pass4(r, kLabels, kUpdMeanOnly, reg, nullptr)) != GMM_OK) return st;
    if ((st = pass4(r, kLabels, kUpdFull, reg, nullptr)) != GMM_OK) return st;
  } else {
    hipLaunchKernelGGL(precompute4_kernel, dim3(1), dim3(kUpdThreads), 0, r.s, w, mu, cov, k,
                       at<float>(ws, r.L.cpar[0]), at<float4>(ws, r.L.shift[0]),
                       at<double>(ws, r.L.th64), at<uint32_t>(ws, r.L.status));
    HIP_TRY(hipGetLastError());
  }
  for (int t = 0; t < opts->iters; ++t) {
    double *slot = loglik ? loglik + t : nullptr;
    if (opts->moment_mode == GMM_MOMENTS_TWO_PASS) {
      if ((st = pass4(r, kSoftStats, kUpdMeanOnly, reg, slot)) != GMM_OK) return st;
      slot = nullptr;
    }
    if ((st = pass4(r, kSoftStats, kUpdFull, reg, slot)) != GMM_OK) return st;
  }
  return pass4(r, kSoftLogLik, kUpdNone, reg, loglik ? loglik + opts->iters : nullptr, w, mu,
               cov);
}

gmm_status finish4(Run4 &r, bool sync) {
  if (!sync) return GMM_OK;
  uint32_t bits = 0;
  HIP_TRY(hipMemcpyAsync(&bits, at<uint32_t>(r.ws, r.L.status), sizeof bits,
                         hipMemcpyDeviceToHost, r.s));
  HIP_TRY(hipStreamSynchronize(r.s));
  return status_from_bits(bits);
}

// ---- captured fits, keyed by every argument the launches depend on
struct Fit4Key {
  const void *pts, *labels, *w, *mu, *cov, *loglik, *ws;
  int64_t n;
  size_t ws_bytes;
  double reg;
  int k, iters, mode, dev;
  const void *tile;
  bool fused, cull;
  const void *ckfn;
  bool operator==(const Fit4Key &o) const {
    return pts == o.pts && labels == o.labels && w == o.w && mu == o.mu && cov == o.cov &&
           loglik == o.loglik && ws == o.ws && n == o.n && ws_bytes == o.ws_bytes &&
           reg == o.reg && k == o.k && iters == o.iters && mode == o.mode && dev == o.dev &&
           tile == o.tile && fused == o.fused && cull == o.cull && ckfn == o.ckfn;
  }
};

struct Graph4Entry {
  bool used = false;
  Fit4Key key{};
  hipGraphExec_t exec = nullptr;
  uint64_t stamp = 0;
};

constexpr int kGraph4Slots = 8;
std::mutex g_graph4_mu;
Graph4Entry g_graph4[kGraph4Slots];
uint64_t g_graph4_clock = 0;

bool graphs_enabled() {
  static int v = -1;
  if (v < 0) {
    const char *e = getenv("GMM_GRAPHS");
    v = (e && e[0] == '0') ? 0 : 1;
  }
  return v == 1;
}

hipStream_t capture_stream4() {
  thread_local hipStream_t cs[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  if (!cs[dev] && hipStreamCreateWithFlags(&cs[dev], hipStreamNonBlocking) != hipSuccess)
    cs[dev] = nullptr;
  return cs[dev];
}

Graph4Entry *graph4_slot(const Fit4Key &key, bool *found) {
  Graph4Entry *victim = &g_graph4[0];
  for (auto &e : g_graph4) {
    if (e.used && e.key == key) {
      *found = true;
      e.stamp = ++g_graph4_clock;
      return &e;
    }
    if (!e.used || (victim->used && e.stamp < victim->stamp)) victim = &e;
  }
  *found = false;
  if (victim->exec) {
    (void)hipDeviceSynchronize();  // an evicted graph may still be running
    (void)hipGraphExecDestroy(victim->exec);
  }
  *victim = Graph4Entry{};
  victim->used = true;
  victim->key = key;
  victim->stamp = ++g_graph4_clock;
  return victim;
}

}  // namespace

extern "C" {

size_t gmm4_fit_workspace_size(int64_t n, int32_t k, const gmm_fit_opts *opts) {
  (void)opts;
  g_err[0] = 0;
  if (check_fit4(n, k) != GMM_OK) return 0;
  Cfg4 c;
  if (!make_cfg4(k, n, &c)) return 0;
  CullCfg4 cc;
  if (cull4_enabled() && !make_cull4(k, n, &cc)) return 0;
  return layout4(k, std::max(c.grid, cc.grid), n, cc.on).total;
}

gmm_status gmm4_fit(const float *pts, int64_t n, int32_t k, const int32_t *init_labels,
                    float *w, float *mu, float *cov, double *loglik,
                    const gmm_fit_opts *opts, void *ws, size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  gmm_status st = check_fit4(n, k);
  if (st != GMM_OK) return st;
  if (!pts || !w || !mu || !cov || !opts) return fail(GMM_ERR_INVALID_ARG, "NULL pointer argument");
  if (reinterpret_cast<uintptr_t>(pts) & 15)
    return fail(GMM_ERR_INVALID_ARG, "points must be 16-byte aligned (N x 4 float32)");
  if (opts->iters < 0) return fail(GMM_ERR_INVALID_ARG, "iters < 0");
  if (!(opts->reg_covar >= 0.0) || !isfinite(opts->reg_covar))
    return fail(GMM_ERR_INVALID_ARG, "reg_covar must be finite and >= 0");
  if (opts->moment_mode != GMM_MOMENTS_SHIFTED && opts->moment_mode != GMM_MOMENTS_TWO_PASS)
    return fail(GMM_ERR_INVALID_ARG, "unknown moment_mode");
  if (opts->flags & ~(GMM_FLAG_ASYNC | GMM_FLAG_DETERMINISTIC))
    return fail(GMM_ERR_INVALID_ARG, "unknown flags");
  if (opts->tol != 0.0) return fail(GMM_ERR_INVALID_ARG, "4D fits run a fixed T (tol = 0)");
  Run4 r;
  r.K = k;
  r.n = n;
  if (!make_cfg4(k, n, &r.c)) return fail(GMM_ERR_UNSUPPORTED, "no 4D launch configuration for k=%d", k);
  if (cull4_enabled() && !make_cull4(k, n, &r.cc))
    return fail(GMM_ERR_UNSUPPORTED, "no culled 4D launch configuration for k=%d", k);
  r.L = layout4(k, std::max(r.c.grid, r.cc.grid), n, r.cc.on);
  r.s = static_cast<hipStream_t>(stream);
  WsGuard guard;
  if ((st = get_ws(&ws, &ws_bytes, r.L.total, r.s, &guard)) != GMM_OK) return st;
  r.ws = ws;
  r.pts = reinterpret_cast<const float4 *>(pts);
  r.labels = init_labels;
  {
    // lambda > 0: the fused reduction + M-step (GMM_FUSED=0 keeps two launches)
    const char *e = getenv("GMM_FUSED");
    r.fused = opts->reg_covar > 0.0 && !(e && e[0] == '0');
  }
  const bool sync = !(opts->flags & GMM_FLAG_ASYNC);
  // repeated calls with the same arguments replay a captured graph (the
  // first runs directly, the second captures); not with a temporary workspace
  if (graphs_enabled() && !guard.ptr) {
    Fit4Key key{pts, init_labels, w, mu, cov, loglik, ws, n, ws_bytes, opts->reg_covar,
                k, opts->iters, opts->moment_mode, 0, r.c.kfn, r.fused, r.cc.on, r.cc.kfn};
    (void)hipGetDevice(&key.dev);
    std::lock_guard<std::mutex> lk(g_graph4_mu);
    bool found = false;
    Graph4Entry *e = graph4_slot(key, &found);
    if (found && !e->exec) {
      hipStream_t cs = capture_stream4();
      if (cs && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        Run4 rc = r;
        rc.s = cs;
        gmm_status cst = enqueue4(rc, w, mu, cov, loglik, opts);
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(cs, &g);
        if (cst == GMM_OK && ee == hipSuccess && g &&
            hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0) != hipSuccess)
          e->exec = nullptr;
        if (g) (void)hipGraphDestroy(g);
      }
      (void)hipGetLastError();
    }
    if (e->exec) {
      HIP_TRY(hipGraphLaunch(e->exec, r.s));
      return finish4(r, sync);
    }
  }
  if ((st = enqueue4(r, w, mu, cov, loglik, opts)) != GMM_OK) return st;
  return finish4(r, sync);
}

size_t gmm4_color_conditional_workspace_size(int32_t k) {
  g_err[0] = 0;
  if (k <= 0 || k > kMaxK) return 0;
  return align256(256) + align256((size_t)k * kCond * sizeof(float));
}

gmm_status gmm4_color_conditional(const float *locs, int64_t m, int32_t k, const float *w,
                                  const float *mu, const float *cov, float *expected,
                                  float *variance, void *ws, size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  if (m <= 0 || m > GMM_MAX_N) return fail(GMM_ERR_INVALID_ARG, "m=%lld out of range", (long long)m);
  if (k <= 0) return fail(GMM_ERR_INVALID_ARG, "k=%d must be positive", k);
  if (k > kMaxK) return fail(GMM_ERR_UNSUPPORTED, "k=%d above the 4D limit %d", k, kMaxK);
  if (!locs || !w || !mu || !cov || !expected || !variance)
    return fail(GMM_ERR_INVALID_ARG, "NULL pointer argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  WsGuard guard;
  gmm_status st = get_ws(&ws, &ws_bytes, gmm4_color_conditional_workspace_size(k), s, &guard);
  if (st != GMM_OK) return st;
  uint32_t *status = at<uint32_t>(ws, 0);
  float *cb = at<float>(ws, align256(256));
  hipLaunchKernelGGL(init4_kernel, dim3(1), dim3(64), 0, s, status, nullptr, 0);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(cond_prep_kernel, dim3(1), dim3(kUpdThreads), 0, s, w, mu, cov, k, cb,
                     status);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(cond4_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, locs, m,
                     cb, k, expected, variance, status);
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

size_t gmm4_joint_dist_sample_workspace_size(int32_t k) {
  g_err[0] = 0;
  if (k <= 0 || k > GMM_MAX_K) return 0;
  return align256(256) + align256((size_t)k * sizeof(double)) +
         align256((size_t)k * 10 * sizeof(double)) + align256(sizeof(int));
}

gmm_status gmm4_joint_dist_sample(int32_t k, const float *w, const float *mu, const float *cov,
                                  int64_t m, const double *u, const float *z, float *out,
                                  int32_t *comp, void *ws, size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  if (m <= 0 || m > GMM_MAX_N) return fail(GMM_ERR_INVALID_ARG, "m=%lld out of range", (long long)m);
  if (k <= 0) return fail(GMM_ERR_INVALID_ARG, "k=%d must be positive", k);
  if (k > GMM_MAX_K) return fail(GMM_ERR_UNSUPPORTED, "k=%d above GMM_MAX_K", k);
  if (!w || !mu || !cov || !u || !z || !out) return fail(GMM_ERR_INVALID_ARG, "NULL pointer argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  WsGuard guard;
  gmm_status st = get_ws(&ws, &ws_bytes, gmm4_joint_dist_sample_workspace_size(k), s, &guard);
  if (st != GMM_OK) return st;
  size_t o = 0;
  uint32_t *status = at<uint32_t>(ws, o); o = align256(o + 256);
  double *run = at<double>(ws, o); o = align256(o + (size_t)k * sizeof(double));
  double *Lf = at<double>(ws, o); o = align256(o + (size_t)k * 10 * sizeof(double));
  int *last = at<int>(ws, o);
  hipLaunchKernelGGL(init4_kernel, dim3(1), dim3(64), 0, s, status, nullptr, 0);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(sample_prep_kernel, dim3(1), dim3(256), 0, s, w, cov, k, run, Lf, last,
                     status);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(sample4_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, run, Lf,
                     last, mu, k, m, u, z, out, comp, status);
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

}  // extern "C"
