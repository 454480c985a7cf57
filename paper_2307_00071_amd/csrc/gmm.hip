// MI355X (gfx950) Gaussian-mixture EM: host side and the C ABI of
// include/gmm.h.  The kernels live in em_device.hpp; one EM iteration is one
// launch of em_tile_kernel (E-step, M-step statistics, cross-block reduction
// and FP64 M-step update).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "em_device.hpp"
#include "small_fit_device.hpp"
#include "order_device.hpp"
#include "kinit_device.hpp"
#include "gmm.h"

// Text of the last host-side error of this thread (shared by every
// translation unit of the library; gmm_last_error returns it).
namespace gmm_host {
thread_local char g_err[512];
}

namespace {

using namespace gmm_dev;
using gmm_host::g_err;

// ======================================================================= host

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
// statistics launches wait in `pending` until gmm_profile_read.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  int reps = 1;
};

// The events skip the system-scope release fence a default event adds at
// its record: that fence writes back L2 and would be timed with the kernel.
bool make_pair(EventPair *p) {
  const unsigned fl = hipEventDisableSystemFence;
  if (hipEventCreateWithFlags(&p->a, fl) != hipSuccess) return false;
  if (hipEventCreateWithFlags(&p->b, fl) != hipSuccess) {
    (void)hipEventDestroy(p->a);
    return false;
  }
  return true;
}

void destroy_pairs(std::vector<EventPair> &v) {
  for (auto &p : v) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  v.clear();
}

struct Profiler {
  int reps = 0;  // tile launches per timed pass; 0 = off
  double ms_total = 0.0;
  int64_t launches = 0;
  std::vector<EventPair> pending;
  // (tile, component) pairs of the timed launches: all, and those the dense
  // kernel evaluated; the culled kernel adds its own to a device counter
  int64_t pairs_all = 0, pairs_dense = 0;
  unsigned long long *dpairs = nullptr;
  int dpairs_dev = -1;
};
thread_local Profiler g_prof;

// Adds the elapsed time of recorded pairs to the totals (waits for them).
hipError_t add_elapsed(const std::vector<EventPair> &v) {
  for (const auto &p : v) {
    hipError_t e = hipEventSynchronize(p.b);
    if (e != hipSuccess) return e;
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess) return e;
    g_prof.ms_total += ms;
    g_prof.launches += p.reps;
  }
  return hipSuccess;
}

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
  int block = 0, tile = 0, grid = 0, P = 0, trip = 0, KC = 0, nch = 0;
  size_t lds = 0;
  void (*launch)(const TileCfg &, hipStream_t, const float4 *, const float *,
                 const float4 *, double *, float *, const TileArgs &) = nullptr;
};

template <int BLOCK, int T, int NCH, int TRIP>
void launch_tile(const TileCfg &c, hipStream_t s, const float4 *pts,
                 const float *cpar, const float4 *shift, double *part,
                 float *lse, const TileArgs &a) {
  hipLaunchKernelGGL((em_tile_kernel<BLOCK, T, NCH, TRIP>), dim3(c.grid),
                     dim3(BLOCK), c.lds, s, pts, cpar, shift, part, lse, a);
}

using LaunchFn = decltype(TileCfg::launch);

// Kernel instances: one per (block, chunks, trip) in use.
template <int BLOCK, int T, int NCH>
bool tile_instance(int trip, LaunchFn *fn, const void **kfn) {
#define GMM_TRIP_CASE(TR)                                                     \
  case TR:                                                                   \
    *fn = &launch_tile<BLOCK, T, NCH, TR>;                                   \
    *kfn = reinterpret_cast<const void *>(&em_tile_kernel<BLOCK, T, NCH, TR>); \
    return true;
  if constexpr (NCH > 1) {
    switch (trip) { GMM_TRIP_CASE(32) GMM_TRIP_CASE(64) default: return false; }
  } else if constexpr (T == 128) {
    switch (trip) {
      GMM_TRIP_CASE(4) GMM_TRIP_CASE(8) GMM_TRIP_CASE(13) GMM_TRIP_CASE(16)
      GMM_TRIP_CASE(26) GMM_TRIP_CASE(32) GMM_TRIP_CASE(64)
      default: return false;
    }
  } else {
    switch (trip) {
      GMM_TRIP_CASE(1) GMM_TRIP_CASE(2) GMM_TRIP_CASE(4) GMM_TRIP_CASE(5)
      GMM_TRIP_CASE(8) GMM_TRIP_CASE(13) GMM_TRIP_CASE(16) GMM_TRIP_CASE(32)
      GMM_TRIP_CASE(64)
      default: return false;
    }
  }
#undef GMM_TRIP_CASE
}

// Largest P <= pmax whose ceil(T/P) consecutive points per subset fit the
// T + 1 entries of an LDS row (so the last subset reads only the zero pad).
int pick_subsets(int pmax, int T) {
  const int TS = T + (T == 64 ? 1 : 3);   // TileShape<., T>::TS
  for (int P = std::min(pmax, T); P >= 1; --P) {
    int trip = (T + P - 1) / P;
    if (P * trip <= TS) return P;
  }
  return 1;
}

template <int BLOCK, int T, int NCH>
bool make_cfg(int K, int64_t n, TileCfg *out) {
  DevInfo di = dev_info();
  if (di.cus <= 0) return false;
  const int KC = (K + NCH - 1) / NCH;
  if (KC > BLOCK) return false;
  const size_t lds = tile_lds_bytes<BLOCK, T>(K, KC);
  const size_t lds_cap = di.lds_max ? di.lds_max : 65536;
  if (lds > lds_cap) return false;
  const int P = pick_subsets(BLOCK / KC, T);
  const int trip = (T + P - 1) / P;
  LaunchFn launch = nullptr;
  const void *fn = nullptr;
  if (!tile_instance<BLOCK, T, NCH>(trip, &launch, &fn)) return false;
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
  const int64_t ntiles = (n + T - 1) / T;
  const int64_t grid = std::min<int64_t>(ntiles, (int64_t)di.cus * per_cu);
  out->block = BLOCK;
  out->tile = T;
  out->grid = (int)grid;
  out->KC = KC;
  out->nch = NCH;
  out->P = P;
  out->trip = trip;
  out->lds = lds;
  out->launch = launch;
  return true;
}

// Launch configuration of the backward kernel (all K components in LDS).
struct BwdCfg {
  int block = 0, tile = 0, grid = 0, P = 0, trip = 0;
  size_t lds = 0;
  void (*launch)(const BwdCfg &, hipStream_t, const float4 *, const float *,
                 const float4 *, const float *, const double *, double *,
                 float *, const TileArgs &, int64_t) = nullptr;
};

template <int BLOCK, int T, int TRIP>
void launch_bwd(const BwdCfg &c, hipStream_t s, const float4 *pts,
                const float *cpar, const float4 *shift, const float *Rt,
                const double *grad_L, double *part, float *g_pts,
                const TileArgs &a, int64_t n) {
  hipLaunchKernelGGL((em_bwd_kernel<BLOCK, T, TRIP>), dim3(c.grid), dim3(BLOCK),
                     c.lds, s, pts, cpar, shift, Rt, grad_L, part, g_pts, a, n);
}

template <int BLOCK, int T>
bool make_bwd_cfg(int K, int64_t n, BwdCfg *out) {
  DevInfo di = dev_info();
  if (di.cus <= 0 || K > BLOCK) return false;
  const size_t lds = bwd_lds_bytes<BLOCK, T>(K);
  if (lds > (di.lds_max ? di.lds_max : 65536)) return false;
  const int P = pick_subsets(BLOCK / K, T);
  const int trip = (T + P - 1) / P;
  const void *fn = nullptr;
  decltype(BwdCfg::launch) launch = nullptr;
#define GMM_BWD_CASE(TR)                                                        \
  case TR:                                                                     \
    launch = &launch_bwd<BLOCK, T, TR>;                                        \
    fn = reinterpret_cast<const void *>(&em_bwd_kernel<BLOCK, T, TR>);         \
    break;
  switch (trip) {
    GMM_BWD_CASE(1) GMM_BWD_CASE(2) GMM_BWD_CASE(4) GMM_BWD_CASE(5)
    GMM_BWD_CASE(8) GMM_BWD_CASE(13) GMM_BWD_CASE(16) GMM_BWD_CASE(32)
    GMM_BWD_CASE(64)
    default: return false;
  }
#undef GMM_BWD_CASE
  if (lds > 65536 &&
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return false;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BLOCK, lds) !=
          hipSuccess || per_cu <= 0)
    return false;
  const int64_t ntiles = (n + T - 1) / T;
  out->block = BLOCK;
  out->tile = T;
  out->grid = (int)std::min<int64_t>(ntiles, (int64_t)di.cus * per_cu);
  out->P = P;
  out->trip = trip;
  out->lds = lds;
  out->launch = launch;
  return true;
}

bool pick_bwd_cfg(int K, int64_t n, BwdCfg *out) {
  if (K <= 128 && make_bwd_cfg<512, 64>(K, n, out)) return true;
  return make_bwd_cfg<1024, 64>(K, n, out);
}

bool reduce_kernel_ready(int K) {
  const size_t lds = update_lds_bytes(K);
  if (lds <= 65536) return true;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(&update_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds) == hipSuccess;
}

// Tile shapes the library can run; the heuristic order is the fallback
// when a shape has not been tuned.  Candidate 0..kNumCand-1.
using MakeCfg = bool (*)(int, int64_t, TileCfg *);
constexpr int kNumCand = 6;
const MakeCfg kCand[kNumCand] = {
    &make_cfg<512, 64, 1>,  &make_cfg<1024, 128, 1>, &make_cfg<512, 128, 1>,
    &make_cfg<256, 64, 1>,  &make_cfg<1024, 64, 1>,  &make_cfg<1024, 64, 2>};
const char *const kCandName[kNumCand] = {"b512t64", "b1024t128", "b512t128",
                                         "b256t64", "b1024t64", "b1024t64c2"};

int default_candidate(int K, int64_t n) {
  TileCfg c;
  if (K <= 128 && kCand[0](K, n, &c)) return 0;
  if (kCand[4](K, n, &c)) return 4;
  if (kCand[5](K, n, &c)) return 5;
  return -1;
}

// ---- autotuner: per (device arch, K, N bucket) the fastest candidate by a
// timed E+M pass on the caller's data at the first call; optional file cache
// (GMM_AUTOTUNE_CACHE).  Enabled by gmm_set_autotune(1) or GMM_AUTOTUNE=1.
struct TuneEntry {
  int K = 0, nb = 0, dev = -1, cand = -1;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
int g_autotune = -1;   // -1: read the environment on first use
bool g_tune_loaded = false;

int n_bucket(int64_t n) {
  int b = 0;
  while ((int64_t)1 << (b + 1) <= n) ++b;
  return b;
}

bool autotune_on() {
  if (g_autotune < 0) {
    const char *e = getenv("GMM_AUTOTUNE");
    g_autotune = (e && e[0] == '1') ? 1 : 0;
  }
  return g_autotune == 1;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = getenv("GMM_AUTOTUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char arch[64], name[64];
  int K, nb;
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t pr;
  const bool have = hipGetDeviceProperties(&pr, dev) == hipSuccess;
  while (fscanf(f, "%63s %d %d %63s", arch, &K, &nb, name) == 4) {
    if (!have || strncmp(arch, pr.gcnArchName, strlen(arch)) != 0) continue;
    for (int i = 0; i < kNumCand; ++i)
      if (strcmp(name, kCandName[i]) == 0) g_tune.push_back(TuneEntry{K, nb, dev, i});
  }
  fclose(f);
}

int tuned_candidate(int K, int64_t n) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int nb = n_bucket(n);
  for (const auto &e : g_tune)
    if (e.K == K && e.nb == nb && e.dev == dev) return e.cand;
  return -1;
}

void tune_store(int K, int64_t n, int cand) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int dev = 0;
  (void)hipGetDevice(&dev);
  g_tune.push_back(TuneEntry{K, n_bucket(n), dev, cand});
  const char *path = getenv("GMM_AUTOTUNE_CACHE");
  hipDeviceProp_t pr;
  if (path && hipGetDeviceProperties(&pr, dev) == hipSuccess) {
    FILE *f = fopen(path, "a");
    if (f) {
      char arch[64];
      snprintf(arch, sizeof arch, "%s", pr.gcnArchName);
      char *colon = strchr(arch, ':');
      if (colon) *colon = 0;
      fprintf(f, "%s %d %d %s\n", arch, K, n_bucket(n), kCandName[cand]);
      fclose(f);
    }
  }
}

// GMM_TILE_SHAPE=<name> forces one shape (when it can run this K).
int forced_candidate() {
  const char *e = getenv("GMM_TILE_SHAPE");
  if (!e || !*e) return -1;
  for (int i = 0; i < kNumCand; ++i)
    if (strcmp(e, kCandName[i]) == 0) return i;
  return -1;
}

bool pick_cfg(int K, int64_t n, TileCfg *out) {
  if (!reduce_kernel_ready(K)) return false;
  const int f = forced_candidate();
  if (f >= 0 && kCand[f](K, n, out)) return true;
  const int t = tuned_candidate(K, n);
  if (t >= 0 && kCand[t](K, n, out)) return true;
  const int d = default_candidate(K, n);
  return d >= 0 && kCand[d](K, n, out);
}

// Launch configuration of the culled tile kernel (soft E+M passes).
struct CullCfg {
  int block = 0, tile = 0, trip = 0, grid = 0;
  size_t lds = 0;
  const char *name = "";
  using Launch = void (*)(const CullCfg &, hipStream_t, const float4 *, const float4 *,
                          const float *, const float4 *, double *, float *,
                          const TileArgs &);
  Launch launch = nullptr;        // soft passes
  Launch launch_lab = nullptr;    // label passes
  Launch launch_means = nullptr;  // soft passes for N and S1 only
};

template <int BLOCK, int T, int TRIP, int SCAP, bool CPR, bool LAB, bool MEANS>
void launch_cull(const CullCfg &c, hipStream_t s, const float4 *pts,
                 const float4 *sph, const float *cpar, const float4 *shift,
                 double *part, float *lse, const TileArgs &a) {
  hipLaunchKernelGGL((em_cull_kernel<BLOCK, T, TRIP, SCAP, CPR, LAB, MEANS>), dim3(c.grid),
                     dim3(BLOCK), c.lds, s, pts, sph, cpar, shift, part, lse, a);
}

template <int BLOCK, int T, int TRIP, int SCAP, bool CPR = false>
bool make_cull_cfg(int K, int64_t n, CullCfg *out) {
  DevInfo di = dev_info();
  if (di.cus <= 0 || K > BLOCK) return false;  // one 64-component chunk per wave
  const size_t lds = cull_lds_bytes<BLOCK, T, TRIP, SCAP, CPR>(K);
  if (lds > (di.lds_max ? di.lds_max : 65536)) return false;
  const void *fn =
      reinterpret_cast<const void *>(&em_cull_kernel<BLOCK, T, TRIP, SCAP, CPR, false, false>);
  const void *fl =
      reinterpret_cast<const void *>(&em_cull_kernel<BLOCK, T, TRIP, SCAP, CPR, true, false>);
  const void *fm =
      reinterpret_cast<const void *>(&em_cull_kernel<BLOCK, T, TRIP, SCAP, CPR, false, true>);
  if (lds > 65536)
    for (const void *f : {fn, fl, fm})
      if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
          hipSuccess)
        return false;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BLOCK, lds) !=
          hipSuccess || per_cu <= 0)
    return false;
  const int64_t ntiles = (n + T - 1) / T;
  out->block = BLOCK;
  out->tile = T;
  out->trip = TRIP;
  out->grid = (int)std::min<int64_t>(ntiles, (int64_t)di.cus * per_cu);
  // GMM_CULL_GRID=<blocks>: fewer persistent blocks (tuning experiments)
  if (const char *g = getenv("GMM_CULL_GRID")) {
    const int v = atoi(g);
    if (v > 0 && v < out->grid) out->grid = v;
  }
  out->lds = lds;
  out->launch = &launch_cull<BLOCK, T, TRIP, SCAP, CPR, false, false>;
  out->launch_lab = &launch_cull<BLOCK, T, TRIP, SCAP, CPR, true, false>;
  out->launch_means = &launch_cull<BLOCK, T, TRIP, SCAP, CPR, false, true>;
  return true;
}

// Shapes: block, tile, points per M-phase lane, E rows kept; "r": cull
// parameters in registers and shifts from global memory (frees 64 B of LDS
// per component).
using MakeCull = bool (*)(int, int64_t, CullCfg *);
constexpr int kNumCull = 14;
const MakeCull kCull[kNumCull] = {
    &make_cull_cfg<512, 128, 16, 64>,        &make_cull_cfg<512, 256, 16, 32>,
    &make_cull_cfg<512, 128, 16, 32>,        &make_cull_cfg<1024, 128, 16, 64>,
    &make_cull_cfg<512, 128, 8, 32>,         &make_cull_cfg<256, 128, 16, 32>,
    &make_cull_cfg<256, 128, 8, 32>,         &make_cull_cfg<256, 64, 8, 32>,
    &make_cull_cfg<1024, 128, 16, 64, true>, &make_cull_cfg<1024, 128, 16, 32, true>,
    &make_cull_cfg<512, 128, 8, 32, true>,   &make_cull_cfg<1024, 128, 16, 96, true>,
    &make_cull_cfg<1024, 128, 16, 128, true>, &make_cull_cfg<1024, 64, 8, 128, true>};
const char *const kCullName[kNumCull] = {
    "c512t128",    "c512t256",   "c512t128s32",   "c1024t128",
    "c512t128p16", "c256t128",   "c256t128p16",   "c256t64",
    "c1024t128r",  "c1024t128s32r", "c512t128p16r", "c1024t128s96r",
    "c1024t128s128r", "c1024t64r"};

// Culling is on unless GMM_CULL=0 or GMM_TILE_SHAPE names a dense shape.
bool pick_cull_cfg(int K, int64_t n, CullCfg *out) {
  const char *off = getenv("GMM_CULL");
  if (off && off[0] == '0') return false;
  const char *e = getenv("GMM_TILE_SHAPE");
  if (e && *e) {
    for (int i = 0; i < kNumCull; ++i)
      if (strcmp(e, kCullName[i]) == 0) {
        if (!kCull[i](K, n, out)) return false;
        out->name = kCullName[i];
        return true;
      }
    return false;
  }
  // measured: subsets of 8 points up to K = 128, of 16 above (depth frame);
  // beyond K = 512 1024-thread blocks with the cull parameters in registers
  // and 128 E rows (LiDAR scan, K = 1000), fewer rows where LDS is short
  static const int small[2] = {4, 3}, mid[2] = {0, 3}, large[4] = {12, 11, 8, 3};
  const int *order = K <= 128 ? small : K <= 512 ? mid : large;
  const int norder = K <= 512 ? 2 : 4;
  for (int o = 0; o < norder; ++o)
    if (const int i = order[o]; kCull[i](K, n, out)) {
      out->name = kCullName[i];
      return true;
    }
  return false;
}

// GMM_DEBUG=1: the launch configuration of each fit on stderr.
void debug_cfg(const char *what, int K, int64_t n, const char *name, int grid,
               int block, size_t lds) {
  const char *e = getenv("GMM_DEBUG");
  if (!e || e[0] != '1') return;
  fprintf(stderr, "gmm: %s K=%d n=%lld kernel %s grid %d block %d lds %zu\n", what, K,
          (long long)n, name, grid, block, lds);
}

// Largest grid over every runnable candidate: the workspace fits any of them.
int max_grid(int K, int64_t n) {
  int g = 0;
  for (int i = 0; i < kNumCand; ++i) {
    TileCfg c;
    if (kCand[i](K, n, &c)) g = std::max(g, c.grid);
  }
  for (int i = 0; i < kNumCull; ++i) {
    CullCfg c;
    if (kCull[i](K, n, &c)) g = std::max(g, c.grid);
  }
  return g;
}

// Workspace layout: two parameter sets (a pass reads one and its epilogue
// writes the other), the FP64 state, the partial rows and the staged points.
struct WsLayout {
  size_t status, counter, pose64, rt32, cpar[2], shift[2], th64, red, part,
      pts4, tsph, total;
  // spatial ordering (fits): unsorted staging, keys/indices, digit counts
  size_t raw4 = 0, keys[2] = {0, 0}, vals[2] = {0, 0}, hist = 0, dtot = 0, box6 = 0;
  int sort_blocks = 0;
  int64_t npad;
  int ncols, nslots;
};

// Largest point count the fit orders spatially (single-block digit scan).
constexpr int64_t kSortMaxN = (int64_t)1 << 30;

WsLayout ws_layout(int64_t n, int K, const TileCfg &c, int extra_cols = 0,
                   int grid_override = 0, bool with_sort = false) {
  WsLayout L{};
  size_t o = 0;
  L.ncols = kNStat * K + 1 + extra_cols;
  L.nslots = std::max(std::max(c.grid, grid_override), max_grid(K, n));
  L.npad = ((n + 255) / 256) * 256;   // a multiple of every tile size
  L.status = o; o = align256(o + 256);
  // stopping rule state (words 0-3), the one-launch fit's grid barrier
  // ticket and give-up flag (words 4, 5)
  L.counter = o; o = align256(o + 8 * sizeof(unsigned));
  L.pose64 = o; o = align256(o + 32 * sizeof(double));
  L.rt32 = o; o = align256(o + 16 * sizeof(float));
  for (int i = 0; i < 2; ++i) {
    L.cpar[i] = o; o = align256(o + (size_t)(K + 1) * kParStride * sizeof(float));
    L.shift[i] = o; o = align256(o + (size_t)K * sizeof(float4));
  }
  L.th64 = o; o = align256(o + (size_t)K * kTh64Stride * sizeof(double));
  L.red = o; o = align256(o + (size_t)kRedChunks * L.ncols * sizeof(double));
  L.part = o; o = align256(o + (size_t)L.nslots * L.ncols * sizeof(double));
  L.pts4 = o; o = align256(o + (size_t)L.npad * sizeof(float4));
  L.tsph = o; o = align256(o + (size_t)(L.npad / 64) * sizeof(float4));
  if (with_sort && L.npad <= kSortMaxN) {
    L.sort_blocks = (int)((L.npad + kSortChunk - 1) / kSortChunk);
    L.raw4 = o; o = align256(o + (size_t)L.npad * sizeof(float4));
    for (int i = 0; i < 2; ++i) {
      L.keys[i] = o; o = align256(o + (size_t)L.npad * sizeof(unsigned));
      L.vals[i] = o; o = align256(o + (size_t)L.npad * sizeof(unsigned));
    }
    L.hist = o; o = align256(o + (size_t)256 * L.sort_blocks * sizeof(unsigned));
    L.dtot = o; o = align256(o + 256 * sizeof(unsigned));
    L.box6 = o; o = align256(o + (size_t)kBoxBlocks * 6 * sizeof(float));
  }
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
  if (bits & kStDevice) return fail(GMM_ERR_DEVICE, "device: the one-launch fit's grid barrier gave up");
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

gmm_status check_sizes(int64_t n, int32_t k, bool fit) {
  if (n <= 0 || n > GMM_MAX_N) return fail(GMM_ERR_INVALID_ARG, "n=%lld out of range", (long long)n);
  if (k <= 0) return fail(GMM_ERR_INVALID_ARG, "k=%d must be positive", k);
  if (k > GMM_MAX_K) return fail(GMM_ERR_UNSUPPORTED, "k=%d above GMM_MAX_K", k);
  if (fit && k > n) return fail(GMM_ERR_INVALID_ARG, "k=%d > n=%lld", k, (long long)n);
  return GMM_OK;
}

// The state of one call: configuration, layout and the current parameter set.
struct Run {
  TileCfg c;      // dense tile kernel (label passes; all passes without culling)
  CullCfg cc;     // culled tile kernel (soft passes), when `cull`
  bool cull = false;
  WsLayout L;
  void *ws = nullptr;
  hipStream_t s = nullptr;
  int K = 0;
  int cur = 0;   // parameter set the next pass reads
  std::vector<EventPair> *sink = nullptr;  // profiling pairs go here
  bool time_loglik = false;  // also time log-likelihood-only passes
  double tol_abs = 0.0;      // > 0: stopping rule |dL| <= tol_abs
  int64_t n = 0;             // points
  bool fused = false;        // lambda > 0: one reduce + update launch per pass
  int conv_par = 0;          // which flag word holds the current stopping state
  bool small = false;        // soft iterations in one launch (em_small_fit_kernel)
};

// The tile kernel alone (writes the partial rows only).
void launch_tiles(Run &r, const TileCfg &c, int mode, float *lse) {
  const WsLayout &L = r.L;
  TileArgs a;
  a.ntiles = (int)(L.npad / c.tile);
  a.K = r.K;
  a.KC = c.KC;
  a.P = c.P;
  a.mode = mode;
  a.ncols = L.ncols;
  c.launch(c, r.s, at<float4>(r.ws, L.pts4), at<float>(r.ws, L.cpar[r.cur]),
           at<float4>(r.ws, L.shift[r.cur]), at<double>(r.ws, L.part), lse, a);
}

// Autotuning: time every runnable tile shape on an E+M pass of the
// current parameters (which no tile pass modifies) and keep the fastest.
gmm_status autotune(Run &r, int64_t n) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best = -1;
  float best_ms = 0.0f;
  TileCfg best_cfg;
  for (int i = 0; i < kNumCand; ++i) {
    TileCfg c;
    if (!kCand[i](r.K, n, &c)) continue;
    launch_tiles(r, c, kSoftStats, nullptr);   // warm-up
    HIP_TRY(hipEventRecord(e0, r.s));
    for (int rep = 0; rep < 3; ++rep) launch_tiles(r, c, kSoftStats, nullptr);
    HIP_TRY(hipEventRecord(e1, r.s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (best < 0 || ms < best_ms) {
      best = i;
      best_ms = ms;
      best_cfg = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best >= 0) {
    tune_store(r.K, n, best);
    r.c = best_cfg;
  }
  return GMM_OK;
}

// One pass: the tile kernel, then the reduction and the M-step update.
gmm_status run_pass(Run &r, int mode, int umode, double reg, double *loglik_slot,
                    float *lse, float *out_w = nullptr, float *out_mu = nullptr,
                    float *out_cov = nullptr) {
  const WsLayout &L = r.L;
  const bool cull = r.cull;  // label passes too: a tile's components are its labels
  TileArgs a;
  a.ntiles = (int)(L.npad / (cull ? r.cc.tile : r.c.tile));
  a.K = r.K;
  a.KC = r.c.KC;
  a.P = r.c.P;
  a.mode = mode;
  a.ncols = L.ncols;
  // with a tolerance, the soft passes check the converged flag: words 0
  // and 1 of the counter buffer take turns as the current and the next
  // state (a full M-step writes the next), the double at word 2 is L_prev
  unsigned *cbase = at<unsigned>(r.ws, L.counter);
  unsigned *conv = (r.tol_abs > 0.0 && mode == kSoftStats) ? cbase + r.conv_par : nullptr;
  unsigned *conv_next = (conv && umode == kUpdFull) ? cbase + (1 - r.conv_par) : nullptr;
  double *Lprev = conv ? reinterpret_cast<double *>(cbase + 2) : nullptr;
  a.conv = conv;
  const int rows = cull ? r.cc.grid : r.c.grid;  // partial rows written
  const bool fuse = r.fused && reg > 0.0;
  a.cmaj = fuse ? 1 : 0;   // the fused reduction reads a component's sums together
  EventPair pp;
  const bool timed = r.sink && (mode == kSoftStats || r.time_loglik);
  if (timed) {
    if (!make_pair(&pp)) return fail(GMM_ERR_DEVICE, "profiling event allocation failed");
    pp.reps = g_prof.reps;
    r.sink->push_back(pp);
    const int64_t all = (int64_t)g_prof.reps * a.ntiles * r.K;
    g_prof.pairs_all += all;
    if (cull)
      a.pairs = g_prof.dpairs;
    else
      g_prof.pairs_dense += all;
    HIP_TRY(hipEventRecord(pp.a, r.s));
  }
  for (int rep = 0; rep < (timed ? g_prof.reps : 1); ++rep) {
    if (cull)
      (mode == kLabels                                  ? r.cc.launch_lab
       : mode == kSoftStats && umode == kUpdMeanOnly ? r.cc.launch_means
                                                     : r.cc.launch)(
                  r.cc, r.s, at<float4>(r.ws, L.pts4), at<float4>(r.ws, L.tsph),
                  at<float>(r.ws, L.cpar[r.cur]), at<float4>(r.ws, L.shift[r.cur]),
                  at<double>(r.ws, L.part), lse, a);
    else
      r.c.launch(r.c, r.s, at<float4>(r.ws, L.pts4), at<float>(r.ws, L.cpar[r.cur]),
                 at<float4>(r.ws, L.shift[r.cur]), at<double>(r.ws, L.part), lse, a);
    HIP_TRY(hipGetLastError());
  }
  if (timed) HIP_TRY(hipEventRecord(pp.b, r.s));
  const int nxt = 1 - r.cur;
  if (conv_next) r.conv_par = 1 - r.conv_par;
  if (fuse) {
    UpdPtrs q;
    q.red2 = nullptr;
    q.cpar_in = at<float>(r.ws, L.cpar[r.cur]);
    q.shift_in = at<float4>(r.ws, L.shift[r.cur]);
    q.cpar_out = at<float>(r.ws, L.cpar[nxt]);
    q.shift_out = at<float4>(r.ws, L.shift[nxt]);
    q.th64 = at<double>(r.ws, L.th64);
    q.loglik_slot = loglik_slot;
    q.out_w = out_w;
    q.out_mu = out_mu;
    q.out_cov = out_cov;
    q.status = at<uint32_t>(r.ws, L.status);
    q.conv = conv;
    q.conv_next = conv_next;
    q.Lprev = Lprev;
    FuseArgs fa;
    fa.K = r.K;
    fa.ncols = L.ncols;
    fa.nrows = rows;
    fa.mode = mode;
    fa.umode = umode;
    fa.reg = reg;
    // the bound C = -3/2 ln(lambda) - 3/2 ln(2 pi) - ln K: every c_b is at
    // most C + ln K (the largest term of a point's sum at most K in value,
    // the sum at most K^2: no FP32 overflow), and a typical weight 1/K puts
    // c_b - C near 0, where its float32 rounding is smallest
    fa.Ntot = (double)r.n + r.K * kEpsN;
    fa.lnZ = log(fa.Ntot) - 1.5 * log(reg) - log((double)r.K);
    fa.Chdr = (-1.5 * log(reg) - 1.5 * kLn2Pi - log((double)r.K)) * kLog2e;
    fa.tol_abs = r.tol_abs;
    hipLaunchKernelGGL(reduce_update_kernel, dim3(r.K), dim3(kFuseThreads), 0, r.s,
                       at<double>(r.ws, L.part), q, fa);
    HIP_TRY(hipGetLastError());
    if (umode != kUpdNone) r.cur = nxt;
    return GMM_OK;
  }
  const int col0 = (mode == kSoftLogLik) ? kNStat * r.K : 0;
  const int ncx = (L.ncols - col0 + 63) / 64;
  hipLaunchKernelGGL(reduce_rows_kernel<1024>, dim3(ncx, kRedChunksFit), dim3(1024), 0,
                     r.s, at<double>(r.ws, L.part), rows, L.ncols, col0,
                     at<double>(r.ws, L.red), conv);
  HIP_TRY(hipGetLastError());
  UpdPtrs q;
  q.red2 = at<double>(r.ws, L.red);
  q.cpar_in = at<float>(r.ws, L.cpar[r.cur]);
  q.shift_in = at<float4>(r.ws, L.shift[r.cur]);
  q.cpar_out = at<float>(r.ws, L.cpar[nxt]);
  q.shift_out = at<float4>(r.ws, L.shift[nxt]);
  q.th64 = at<double>(r.ws, L.th64);
  q.loglik_slot = loglik_slot;
  q.out_w = out_w;
  q.out_mu = out_mu;
  q.out_cov = out_cov;
  q.status = at<uint32_t>(r.ws, L.status);
  q.conv = conv;
  q.conv_next = conv_next;
  q.Lprev = Lprev;
  UpdArgs ua;
  ua.ncols = L.ncols;
  ua.col0 = col0;
  ua.K = r.K;
  ua.mode = mode;
  ua.umode = umode;
  ua.reg = reg;
  ua.tol_abs = r.tol_abs;
  hipLaunchKernelGGL(update_kernel, dim3(1), dim3(kUpdThreads),
                     update_lds_bytes(r.K), r.s, q, ua);
  HIP_TRY(hipGetLastError());
  if (umode != kUpdNone) r.cur = nxt;
  return GMM_OK;
}

gmm_status run_init(Run &r, bool zero_shift) {
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(256), 0, r.s,
                     at<uint32_t>(r.ws, r.L.status),
                     at<unsigned>(r.ws, r.L.counter), 8,
                     zero_shift ? at<float4>(r.ws, r.L.shift[r.cur]) : nullptr,
                     r.K);
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

gmm_status run_precompute(Run &r, const float *w, const float *mu,
                          const float *cov) {
  hipLaunchKernelGGL(precompute_kernel, dim3(1), dim3(kPreThreads), 0, r.s, w,
                     mu, cov, r.K, at<float>(r.ws, r.L.cpar[r.cur]),
                     at<float4>(r.ws, r.L.shift[r.cur]),
                     at<double>(r.ws, r.L.th64), at<uint32_t>(r.ws, r.L.status));
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

// Morton order of the staged points: raw4 -> pts4 (see order_device.hpp).
gmm_status spatial_order(Run &r, int64_t n) {
  const WsLayout &L = r.L;
  const int64_t npad = L.npad;
  const int nblk = L.sort_blocks;
  hipLaunchKernelGGL(bbox_kernel, dim3(kBoxBlocks), dim3(kSortThreads), 0, r.s,
                     at<float4>(r.ws, L.raw4), n, at<float>(r.ws, L.box6));
  HIP_TRY(hipGetLastError());
  const unsigned mb = (unsigned)std::min<int64_t>(256, (npad + kSortThreads - 1) / kSortThreads);
  hipLaunchKernelGGL(morton_kernel, dim3(mb), dim3(kSortThreads), 0, r.s,
                     at<float4>(r.ws, L.raw4), n, npad, at<float>(r.ws, L.box6),
                     kBoxBlocks, at<unsigned>(r.ws, L.keys[0]),
                     at<unsigned>(r.ws, L.vals[0]));
  HIP_TRY(hipGetLastError());
  int src = 0;
  for (int shift = 0; shift < 24; shift += 8, src = 1 - src) {
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nblk), dim3(kSortThreads), 0, r.s,
                       at<unsigned>(r.ws, L.keys[src]), npad, shift,
                       at<unsigned>(r.ws, L.hist), nblk);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(radix_scan_kernel, dim3(256), dim3(kSortThreads), 0, r.s,
                       at<unsigned>(r.ws, L.hist), nblk, at<unsigned>(r.ws, L.dtot));
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblk), dim3(kSortThreads), 0, r.s,
                       at<unsigned>(r.ws, L.keys[src]), at<unsigned>(r.ws, L.vals[src]),
                       npad, shift, at<unsigned>(r.ws, L.hist), nblk,
                       at<unsigned>(r.ws, L.dtot), at<unsigned>(r.ws, L.keys[1 - src]),
                       at<unsigned>(r.ws, L.vals[1 - src]));
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((npad + kSortThreads - 1) / kSortThreads)),
                     dim3(kSortThreads), 0, r.s, at<float4>(r.ws, L.raw4),
                     at<unsigned>(r.ws, L.vals[src]), npad, at<float4>(r.ws, L.pts4));
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

// Spatial ordering is used by culled fits unless GMM_SORT=0.
bool sort_enabled() {
  const char *e = getenv("GMM_SORT");
  return !(e && e[0] == '0');
}

gmm_status stage(Run &r, const float *pts, int64_t n, const int32_t *labels,
                 const float *Rt, bool sort = false) {
  const int64_t nb = (r.L.npad + 255) / 256;
  sort = sort && r.cull && r.L.sort_blocks > 0;
  hipLaunchKernelGGL(stage_kernel, dim3((unsigned)nb), dim3(256), 0, r.s, pts,
                     n, r.L.npad, labels, r.K, Rt,
                     at<float4>(r.ws, sort ? r.L.raw4 : r.L.pts4),
                     at<uint32_t>(r.ws, r.L.status));
  HIP_TRY(hipGetLastError());
  if (sort) {
    gmm_status st = spatial_order(r, n);
    if (st != GMM_OK) return st;
  }
  if (r.cull) {
    const int64_t nt = r.L.npad / r.cc.tile;
    hipLaunchKernelGGL(tile_sphere_kernel, dim3((unsigned)nt), dim3(256), 0, r.s,
                       at<float4>(r.ws, r.L.pts4), r.cc.tile,
                       at<float4>(r.ws, r.L.tsph));
    HIP_TRY(hipGetLastError());
  }
  return GMM_OK;
}

gmm_status finish(Run &r, bool sync) {
  if (!sync) return GMM_OK;
  uint32_t bits = 0;
  HIP_TRY(hipMemcpyAsync(&bits, at<uint32_t>(r.ws, r.L.status), sizeof bits,
                         hipMemcpyDeviceToHost, r.s));
  HIP_TRY(hipStreamSynchronize(r.s));
  return status_from_bits(bits);
}

// Fits with K <= 16 components and at most 256 tiles of 256 points (and
// no more tiles than compute units) with shifted moments run their soft
// iterations in one launch of em_small_fit_kernel: one block per tile, all
// resident at once.  GMM_SMALL=0, or a tile shape forced by GMM_TILE_SHAPE,
// keeps a launch pair per iteration.
int small_give_up() {
  const char *e = getenv("GMM_SMALL_TEST_GIVE_UP");
  return e ? atoi(e) : -1;
}

bool small_fit_ok(int K, const WsLayout &L, const gmm_fit_opts *opts) {
  const char *e = getenv("GMM_SMALL");
  if ((e && e[0] == '0') || getenv("GMM_TILE_SHAPE")) return false;
  const int64_t nt = L.npad / kSmallThreads;
  return K <= kSmallMaxK && nt <= kSmallMaxTiles && nt <= dev_info().cus &&
         2 * nt <= L.nslots && opts->moment_mode == GMM_MOMENTS_SHIFTED &&
         opts->iters > 0;
}

// The soft iterations of a small fit: parameters cur -> 1 - cur, the
// log-likelihood of iteration t into loglik[t].
gmm_status run_small(Run &r, int iters, double reg, double *loglik) {
  const WsLayout &L = r.L;
  SmallArgs a;
  a.K = r.K;
  int P = 1;   // point subsets: the largest power of two with P K <= 256
  while (2 * P * r.K <= kSmallThreads) P *= 2;
  a.P = P;
  a.trip = kSmallThreads / P;
  a.iters = iters;
  a.ncols = L.ncols;
  a.reg = reg;
  a.tol_abs = r.tol_abs;
  // GMM_SMALL_TEST_GIVE_UP=t: block 0 gives up at the barrier of iteration t
  // (tests of the error path; every block still exits)
  a.give_up_at = small_give_up();
  const int grid = (int)(L.npad / kSmallThreads);
  const int nxt = 1 - r.cur;
  hipLaunchKernelGGL(em_small_fit_kernel, dim3(grid), dim3(kSmallThreads), 0, r.s,
                     at<float4>(r.ws, L.pts4), at<float>(r.ws, L.cpar[r.cur]),
                     at<float4>(r.ws, L.shift[r.cur]), at<float>(r.ws, L.cpar[nxt]),
                     at<float4>(r.ws, L.shift[nxt]), at<double>(r.ws, L.th64),
                     at<double>(r.ws, L.part), at<unsigned>(r.ws, L.counter) + 4,
                     loglik, at<uint32_t>(r.ws, L.status), a);
  HIP_TRY(hipGetLastError());
  r.cur = nxt;
  return GMM_OK;
}

// Every launch of one fit, in order.
gmm_status enqueue_fit(Run &r, const float *pts, int64_t n,
                       const int32_t *init_labels, float *w, float *mu,
                       float *cov, double *loglik, const gmm_fit_opts *opts,
                       bool may_tune) {
  gmm_status st;
  if ((st = run_init(r, init_labels != nullptr)) != GMM_OK) return st;
  if ((st = stage(r, pts, n, init_labels, nullptr, sort_enabled())) != GMM_OK) return st;
  const double reg = opts->reg_covar;
  if (init_labels) {
    // theta_0 = M-step of the one-hot responsibilities, two passes: the mean
    // (shift 0), then the scatter about it.
    if ((st = run_pass(r, kLabels, kUpdMeanOnly, reg, nullptr, nullptr)) != GMM_OK) return st;
    if ((st = run_pass(r, kLabels, kUpdFull, reg, nullptr, nullptr)) != GMM_OK) return st;
  } else {
    if ((st = run_precompute(r, w, mu, cov)) != GMM_OK) return st;
  }
  if (may_tune && !r.cull && !r.small && autotune_on() && forced_candidate() < 0 &&
      tuned_candidate(r.K, n) < 0 &&
      (st = autotune(r, n)) != GMM_OK)
    return st;
  if (r.small) {
    if ((st = run_small(r, opts->iters, reg, loglik)) != GMM_OK) return st;
  } else for (int t = 0; t < opts->iters; ++t) {
    double *slot = loglik ? loglik + t : nullptr;
    if (opts->moment_mode == GMM_MOMENTS_TWO_PASS) {
      if ((st = run_pass(r, kSoftStats, kUpdMeanOnly, reg, slot, nullptr)) != GMM_OK) return st;
      slot = nullptr;
    }
    if ((st = run_pass(r, kSoftStats, kUpdFull, reg, slot, nullptr)) != GMM_OK) return st;
  }
  // log-likelihood of the returned parameters and the FP32 outputs
  return run_pass(r, kSoftLogLik, kUpdNone, reg,
                  loglik ? loglik + opts->iters : nullptr, nullptr, w, mu, cov);
}

// Argument checks, launch configuration and workspace layout of a fit.
gmm_status fit_setup(const float *pts, int64_t n, int32_t k, const float *w,
                     const float *mu, const float *cov, const gmm_fit_opts *opts,
                     void *stream, Run *r) {
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
  if (opts->flags & ~(GMM_FLAG_ASYNC | GMM_FLAG_DETERMINISTIC))
    return fail(GMM_ERR_INVALID_ARG, "unknown flags");
  if (!(opts->tol >= 0.0) || !isfinite(opts->tol))
    return fail(GMM_ERR_INVALID_ARG, "tol must be finite and >= 0");
  r->tol_abs = opts->tol * (double)n;
  r->n = n;
  // lambda > 0: the fused reduction + M-step (GMM_FUSED=0 keeps two launches)
  {
    const char *e = getenv("GMM_FUSED");
    r->fused = opts->reg_covar > 0.0 && !(e && e[0] == '0');
  }
  r->K = k;
  if (!pick_cfg(k, n, &r->c)) return fail(GMM_ERR_UNSUPPORTED, "no launch configuration for k=%d", k);
  r->cull = pick_cull_cfg(k, n, &r->cc);
  if (r->cull) debug_cfg("fit", k, n, r->cc.name, r->cc.grid, r->cc.block, r->cc.lds);
  r->L = ws_layout(n, k, r->c, 0, 0, true);
  // a one-launch fit runs its label and final passes dense: the spatial
  // order and the tile spheres of culling would cost more than they save.
  // Profiled fits (per-pass tile timing) keep the launch pairs.
  r->small = g_prof.reps == 0 && small_fit_ok(k, r->L, opts);
  if (r->small) r->cull = false;
  r->s = static_cast<hipStream_t>(stream);
  return GMM_OK;
}

// ------------------------------------------------------------ graph cache
// A fit repeated with identical arguments (same buffers, sizes, options and
// workspace) is captured once into a hipGraph on a private stream and then
// replayed on the caller's stream: T iterations become one submission.  The
// first call with a new argument set runs directly; the second captures.
struct FitKey {
  const void *pts, *labels, *w, *mu, *cov, *loglik, *ws;
  int64_t n;
  size_t ws_bytes;
  double reg, tol;
  int k, iters, mode, dev;
  const void *dense, *culled;  // the kernels the fit launches
  bool sorted, fused, small;
  int give_up;   // GMM_SMALL_TEST_GIVE_UP (a launch argument)
  bool operator==(const FitKey &o) const {
    return pts == o.pts && labels == o.labels && w == o.w && mu == o.mu &&
           cov == o.cov && loglik == o.loglik && ws == o.ws && n == o.n &&
           ws_bytes == o.ws_bytes && reg == o.reg && tol == o.tol && k == o.k &&
           iters == o.iters && mode == o.mode && dev == o.dev &&
           dense == o.dense && culled == o.culled && sorted == o.sorted &&
           fused == o.fused && small == o.small && give_up == o.give_up;
  }
};

struct GraphEntry {
  bool used = false;
  FitKey key{};
  hipGraphExec_t exec = nullptr;
  uint64_t stamp = 0;
};

constexpr int kGraphSlots = 8;
std::mutex g_graph_mu;
GraphEntry g_graphs[kGraphSlots];
uint64_t g_graph_clock = 0;

bool graphs_enabled() {
  static int v = -1;
  if (v < 0) {
    const char *e = getenv("GMM_GRAPHS");
    v = (e && e[0] == '0') ? 0 : 1;
  }
  return v == 1;
}

hipStream_t capture_stream() {
  thread_local hipStream_t cs[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  if (!cs[dev] && hipStreamCreateWithFlags(&cs[dev], hipStreamNonBlocking) != hipSuccess)
    cs[dev] = nullptr;
  return cs[dev];
}

void release_entry(GraphEntry &e) {
  if (e.exec) {
    (void)hipDeviceSynchronize();  // an evicted graph may still be running
    (void)hipGraphExecDestroy(e.exec);
  }
  e = GraphEntry{};
}

// Returns the slot for key: found (exec set or not), or a fresh one.
GraphEntry *graph_slot(const FitKey &key, bool *found) {
  GraphEntry *victim = &g_graphs[0];
  for (auto &e : g_graphs) {
    if (e.used && e.key == key) {
      *found = true;
      e.stamp = ++g_graph_clock;
      return &e;
    }
    if (!e.used || (victim->used && e.stamp < victim->stamp)) victim = &e;
  }
  *found = false;
  release_entry(*victim);
  victim->used = true;
  victim->key = key;
  victim->stamp = ++g_graph_clock;
  return victim;
}


// ============================================================ batched fits
//
// All frames' points are staged into 64-point tiles, each frame padded to a
// multiple of 128 points (so the culled shapes' 128-point tiles never span
// two frames).  A soft pass launches the tile kernel once per M-phase trip
// class of the dense shapes (frames whose point-subset split gives the same
// TRIP; LDS and grid sized for the class) or once for the culled shapes;
// each launch cuts its frames' tiles into contiguous per-block ranges of
// equal cost (tiles x K_f), split at frame boundaries into segments, and a
// block writes one FP64 partial row per segment it touches.
// reduce_frames_kernel and update_frames_kernel then finish every frame at
// once; the whole T-iteration loop is captured into one hipGraph per call.
// (One dense launch over all frames, with the trip chosen per segment and
// LDS sized for the largest K, measured 3.5 ms per pass on the 64-frame
// workload against about 1.2 ms for the class launches.)
//
// Launch shapes: dense 512- or 1024-thread blocks ("bb512", "bb1024"), or
// the culled kernel (512 threads, 128-point tiles in each frame's own Morton
// order) with (TRIP, SCAP) = (8, 32), (8, 64) or (16, 64).  Label passes
// always use the dense 512 shape (1024 beyond 512 components).  With
// autotuning on, the first batched fit for a new (device, B, K_max,
// log2 sum N_f K_f) runs a few EM iterations, times one soft pass of every
// runnable shape on the caller's own data and keeps the fastest (cached per
// process and in GMM_AUTOTUNE_CACHE); GMM_BATCH_SHAPE forces a shape;
// GMM_BATCH_CULL=1 selects the first culled shape; the default is the dense
// 512 shape.

constexpr int kBatchT = 64;        // dense tiles
constexpr int kBatchTuneIters = 4; // EM iterations before the shapes are timed
constexpr int kBatchCullT = 128;   // culled tiles; every frame is padded to this
constexpr int kBatchMaxK = 512;    // largest K_f

// One launch of a batched pass: its frames' segments (cost-balanced block
// ranges), grid, LDS and kernel instance.
struct BatchLaunchSet;
using BatchLaunch = void (*)(const BatchLaunchSet &, hipStream_t, const float4 *,
                             const float4 *, const float *, const float4 *, double *,
                             const unsigned char *, size_t frames_off, int);

struct BatchLaunchSet {
  int trip = 0, kc_max = 0, grid = 0;
  size_t lds = 0;
  BatchLaunch launch = nullptr;
  std::vector<BSeg> segs;
  std::vector<int> blk;         // grid + 1 segment offsets
  size_t seg_off = 0, blk_off = 0;   // in the plan upload
};

// A launch shape of the batched soft pass over every frame: the dense
// kernel takes one launch per M-phase trip class (frames whose point-subset
// split gives the same TRIP, LDS sized for the class's largest K), the
// culled kernel one launch.
struct BatchVariant {
  int spec = -1;
  std::vector<BFrame> frames;   // this shape's P, nrows and poff per frame
  size_t frames_off = 0;
  std::vector<BatchLaunchSet> sets;
  int64_t part_len = 0;
};

template <int BLOCK, int TRIP>
void launch_batch_dense(const BatchLaunchSet &c, hipStream_t s, const float4 *pts,
                        const float4 *, const float *cpar, const float4 *shift,
                        double *part, const unsigned char *plan, size_t frames_off, int mode) {
  hipLaunchKernelGGL((em_batch_kernel<BLOCK, kBatchT, TRIP>), dim3(c.grid), dim3(BLOCK), c.lds,
                     s, pts, cpar, shift, part,
                     reinterpret_cast<const BFrame *>(plan + frames_off),
                     reinterpret_cast<const BSeg *>(plan + c.seg_off),
                     reinterpret_cast<const int *>(plan + c.blk_off), mode, c.kc_max);
}

template <int TRIP, int SCAP>
void launch_batch_cull(const BatchLaunchSet &c, hipStream_t s, const float4 *pts,
                       const float4 *sph, const float *cpar, const float4 *shift,
                       double *part, const unsigned char *plan, size_t frames_off, int mode) {
  hipLaunchKernelGGL((em_cull_batch_kernel<512, kBatchCullT, TRIP, SCAP>), dim3(c.grid),
                     dim3(512), c.lds, s, pts, sph, cpar, shift, part,
                     reinterpret_cast<const BFrame *>(plan + frames_off),
                     reinterpret_cast<const BSeg *>(plan + c.seg_off),
                     reinterpret_cast<const int *>(plan + c.blk_off), mode, c.kc_max);
}

// The dense kernel instance of (BLOCK, TRIP): launcher and function.
template <int BLOCK>
bool dense_instance(int trip, BatchLaunch *fn, const void **kfn) {
#define GMM_BATCH_CASE(TR)                                                             \
  case TR:                                                                            \
    *fn = &launch_batch_dense<BLOCK, TR>;                                              \
    *kfn = reinterpret_cast<const void *>(&em_batch_kernel<BLOCK, kBatchT, TR>);       \
    return true;
  switch (trip) {
    GMM_BATCH_CASE(1) GMM_BATCH_CASE(2) GMM_BATCH_CASE(4) GMM_BATCH_CASE(5)
    GMM_BATCH_CASE(8) GMM_BATCH_CASE(13) GMM_BATCH_CASE(16) GMM_BATCH_CASE(32)
    GMM_BATCH_CASE(64)
    default: return false;
  }
#undef GMM_BATCH_CASE
}

struct BatchSpec {
  const char *name;
  bool cull;
  int block, tile;
  // dense: the instance of a trip; culled: the one instance
  bool (*instance)(int trip, BatchLaunch *fn, const void **kfn);
  size_t (*lds)(int kmax);
};

template <int TRIP, int SCAP>
bool cull_instance(int, BatchLaunch *fn, const void **kfn) {
  *fn = &launch_batch_cull<TRIP, SCAP>;
  *kfn = reinterpret_cast<const void *>(&em_cull_batch_kernel<512, kBatchCullT, TRIP, SCAP>);
  return true;
}

size_t lds_dense512(int k) { return batch_lds_bytes<512, kBatchT>(k); }
size_t lds_dense1024(int k) { return batch_lds_bytes<1024, kBatchT>(k); }
size_t lds_c8s32(int k) { return cull_lds_bytes<512, kBatchCullT, 8, 32>(k); }
size_t lds_c8s64(int k) { return cull_lds_bytes<512, kBatchCullT, 8, 64>(k); }
size_t lds_c16s64(int k) { return cull_lds_bytes<512, kBatchCullT, 16, 64>(k); }

constexpr int kNumBatchSpec = 5;
const BatchSpec kBatchSpec[kNumBatchSpec] = {
    {"bb512", false, 512, kBatchT, &dense_instance<512>, &lds_dense512},
    {"bb1024", false, 1024, kBatchT, &dense_instance<1024>, &lds_dense1024},
    {"bc512p8s32", true, 512, kBatchCullT, &cull_instance<8, 32>, &lds_c8s32},
    {"bc512p8s64", true, 512, kBatchCullT, &cull_instance<8, 64>, &lds_c8s64},
    {"bc512p16s64", true, 512, kBatchCullT, &cull_instance<16, 64>, &lds_c16s64},
};

struct BatchPlan {
  int B = 0, Ktot = 0, Kmax = 0, ncols_max = 0;
  int64_t tiles = 0;   // staged 64-point tiles (frames padded to 128 points)
  int64_t evals = 0;   // sum N_f K_f
  std::vector<BFrame> base;   // frame table of the reductions, updates and sort
  std::vector<BatchVariant> vars;
  int lab_var = -1, soft_var = -1;
  bool sort = false;          // a culled shape is present: Morton order + spheres
  size_t plan_bytes = 0;
  // workspace offsets
  size_t status, plan, cpar[2], shift[2], th64, red, part, pts4, total;
  size_t raw4 = 0, keys[2] = {0, 0}, vals[2] = {0, 0}, hist = 0, dtot = 0, box6 = 0,
         tsph = 0;
  int sort_blocks = 0;
  size_t red_len = 0, part_len = 0;
};

// Cost-balanced contiguous block ranges over the tiles of the frames fr
// (tiles of `tile` points; cost = tiles x K_f), cut at frame boundaries into
// segments; nrows counts each frame's segments (its partial rows).
void cut_segments(const std::vector<BFrame> &frames, const std::vector<int> &fr, int tile,
                  int grid, std::vector<int> &nrows, BatchLaunchSet *c) {
  const int r = tile / kBatchT;
  double cost = 0.0;
  for (int f : fr) cost += (double)((frames[f].n + tile - 1) / tile) * frames[f].K;
  const double target = cost / grid;
  double acc = 0.0;
  int blk = 0;
  c->segs.clear();
  c->blk.assign(1, 0);
  for (int f : fr) {
    const BFrame &F = frames[f];
    const int64_t nt = (F.n + tile - 1) / tile;
    const int64_t t0 = F.toff / r;
    int64_t t = 0;
    while (t < nt) {
      const double room = (blk + 1) * target - acc;
      int64_t take = (int64_t)std::ceil(room / F.K - 1e-9);
      if (blk == grid - 1) take = nt - t;
      take = std::max<int64_t>(1, std::min<int64_t>(take, nt - t));
      c->segs.push_back(BSeg{f, (int)(t0 + t), (int)(t0 + t + take), nrows[f]++});
      t += take;
      acc += (double)take * F.K;
      if (acc >= (blk + 1) * target - 1e-6 && blk < grid - 1) {
        ++blk;
        c->blk.push_back((int)c->segs.size());
      }
    }
  }
  while ((int)c->blk.size() < grid + 1) c->blk.push_back((int)c->segs.size());
}

// One shape over the frames: its frame table (P per frame), launches with
// their segments, and the partial-row layout; false when it cannot run
// these frames.
bool make_variant(const BatchPlan &bp, int spec, int cus, size_t lds_max, BatchVariant *v) {
  const BatchSpec &S = kBatchSpec[spec];
  if (bp.Kmax > (S.cull ? 512 : S.block)) return false;
  v->spec = spec;
  v->frames = bp.base;
  v->sets.clear();
  std::vector<int> trips(bp.B, 0);
  for (int f = 0; f < bp.B; ++f) {
    BFrame &F = v->frames[f];
    F.P = pick_subsets(S.block / F.K, kBatchT);
    trips[f] = S.cull ? 0 : (kBatchT + F.P - 1) / F.P;
  }
  std::vector<int> classes = trips;
  std::sort(classes.begin(), classes.end());
  classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
  std::vector<int> nrows(bp.B, 0);
  for (int tr : classes) {
    BatchLaunchSet c;
    c.trip = tr;
    std::vector<int> fr;
    for (int f = 0; f < bp.B; ++f)
      if (trips[f] == tr) {
        fr.push_back(f);
        c.kc_max = std::max(c.kc_max, v->frames[f].K);
      }
    const void *kfn = nullptr;
    if (!S.instance(tr, &c.launch, &kfn)) return false;
    c.lds = S.lds(c.kc_max);
    if (c.lds > (lds_max ? lds_max : 65536)) return false;
    if (c.lds > 65536 &&
        hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds) !=
            hipSuccess)
      return false;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, S.block, c.lds) !=
            hipSuccess || per_cu <= 0)
      return false;
    int64_t ntile = 0;
    for (int f : fr) ntile += (v->frames[f].n + S.tile - 1) / S.tile;
    c.grid = (int)std::max<int64_t>(1, std::min<int64_t>(ntile, (int64_t)cus * per_cu));
    cut_segments(v->frames, fr, S.tile, c.grid, nrows, &c);
    v->sets.push_back(std::move(c));
  }
  int64_t poff = 0;
  for (int f = 0; f < bp.B; ++f) {
    v->frames[f].nrows = nrows[f];
    v->frames[f].poff = poff;
    poff += (int64_t)nrows[f] * v->frames[f].ncols;
  }
  v->part_len = poff;
  return true;
}

// The frames, the label shape and the soft shape(s): every runnable shape
// when `all` (autotuning and workspace sizing), else the one named by
// soft_spec (-1: the default).
gmm_status make_batch_plan(int B, const int64_t *pt_off, const int32_t *k_off,
                           BatchPlan *bp, bool all, int soft_spec = -1) {
  DevInfo di = dev_info();
  if (di.cus <= 0) return fail(GMM_ERR_DEVICE, "no HIP device");
  if (B <= 0) return fail(GMM_ERR_INVALID_ARG, "B=%d must be positive", B);
  *bp = BatchPlan{};
  bp->B = B;
  bp->base.assign(B, BFrame{});
  int64_t toff = 0;
  int cpoff = 0, roff = 0;
  for (int f = 0; f < B; ++f) {
    const int64_t n = pt_off[f + 1] - pt_off[f];
    const int K = k_off[f + 1] - k_off[f];
    if (n <= 0 || K <= 0 || K > n)
      return fail(GMM_ERR_INVALID_ARG, "frame %d: n=%lld k=%d", f, (long long)n, K);
    if (K > kBatchMaxK) return fail(GMM_ERR_UNSUPPORTED, "frame %d: k=%d above %d", f, K, kBatchMaxK);
    if (n > ((int64_t)1 << 30)) return fail(GMM_ERR_UNSUPPORTED, "frame %d: n=%lld too large", f, (long long)n);
    BFrame &F = bp->base[f];
    F.K = K;
    F.koff = k_off[f] - k_off[0];
    F.cpoff = cpoff;
    cpoff += (K + 1) * kParStride;
    F.ncols = kNStat * K + 1;
    F.roff = roff;
    roff += F.ncols;
    F.toff = toff;
    F.n = (int)n;
    toff += (n + kBatchCullT - 1) / kBatchCullT * (kBatchCullT / kBatchT);
    bp->Kmax = std::max(bp->Kmax, K);
    bp->ncols_max = std::max(bp->ncols_max, F.ncols);
    bp->evals += n * K;
  }
  bp->Ktot = k_off[B] - k_off[0];
  bp->tiles = toff;
  bp->red_len = roff;
  if (toff * kBatchT >= ((int64_t)1 << 31))
    return fail(GMM_ERR_UNSUPPORTED, "%lld staged points above the batched limit", (long long)(toff * kBatchT));
  // label shape: dense 512 (1024 above 512 components)
  const int lab_spec = bp->Kmax <= 512 ? 0 : 1;
  bp->vars.clear();
  BatchVariant lv;
  if (!make_variant(*bp, lab_spec, di.cus, di.lds_max, &lv))
    return fail(GMM_ERR_UNSUPPORTED, "no batched launch configuration for K_max=%d", bp->Kmax);
  bp->vars.push_back(std::move(lv));
  bp->lab_var = 0;
  bp->soft_var = 0;
  const bool cull_ok = [] {
    const char *off = getenv("GMM_CULL");
    return !(off && off[0] == '0');
  }() && B <= 256;
  for (int s = 0; s < kNumBatchSpec; ++s) {
    if (s == lab_spec) continue;
    if (!all && s != soft_spec) continue;
    if (kBatchSpec[s].cull && !cull_ok) continue;
    BatchVariant v;
    if (!make_variant(*bp, s, di.cus, di.lds_max, &v)) continue;
    if (s == soft_spec) bp->soft_var = (int)bp->vars.size();
    bp->vars.push_back(std::move(v));
  }
  for (const auto &v : bp->vars) bp->sort = bp->sort || kBatchSpec[v.spec].cull;
  bp->part_len = 0;
  for (const auto &v : bp->vars) bp->part_len = std::max<int64_t>(bp->part_len, v.part_len);
  // plan upload: the base frame table, then each shape's tables
  size_t o = align256(sizeof(BFrame) * B);
  for (auto &v : bp->vars) {
    v.frames_off = o; o = align256(o + sizeof(BFrame) * B);
    for (auto &c : v.sets) {
      c.seg_off = o; o = align256(o + sizeof(BSeg) * c.segs.size());
      c.blk_off = o; o = align256(o + sizeof(int) * c.blk.size());
    }
  }
  bp->plan_bytes = o;
  // workspace
  o = 0;
  bp->status = o; o = align256(o + 256);
  bp->plan = o; o = align256(o + bp->plan_bytes);
  const size_t npar = (size_t)(bp->Ktot + B) * kParStride;
  for (int i = 0; i < 2; ++i) {
    bp->cpar[i] = o; o = align256(o + npar * sizeof(float));
    bp->shift[i] = o; o = align256(o + (size_t)bp->Ktot * sizeof(float4));
  }
  bp->th64 = o; o = align256(o + (size_t)bp->Ktot * kTh64Stride * sizeof(double));
  bp->red = o; o = align256(o + bp->red_len * sizeof(double));
  bp->part = o; o = align256(o + bp->part_len * sizeof(double));
  bp->pts4 = o; o = align256(o + (size_t)bp->tiles * kBatchT * sizeof(float4));
  if (bp->sort) {
    const size_t np = (size_t)bp->tiles * kBatchT;
    bp->tsph = o; o = align256(o + np / kBatchCullT * sizeof(float4));
    bp->sort_blocks = (int)((np + kSortChunk - 1) / kSortChunk);
    bp->raw4 = o; o = align256(o + np * sizeof(float4));
    for (int i = 0; i < 2; ++i) {
      bp->keys[i] = o; o = align256(o + np * sizeof(unsigned));
      bp->vals[i] = o; o = align256(o + np * sizeof(unsigned));
    }
    bp->hist = o; o = align256(o + (size_t)256 * bp->sort_blocks * sizeof(unsigned));
    bp->dtot = o; o = align256(o + 256 * sizeof(unsigned));
    bp->box6 = o; o = align256(o + (size_t)B * 6 * sizeof(float));
  }
  bp->total = o;
  return GMM_OK;
}

int batch_spec_by_name(const char *name) {
  for (int s = 0; s < kNumBatchSpec; ++s)
    if (strcmp(kBatchSpec[s].name, name) == 0) return s;
  return -1;
}

// The soft shape a call would use without tuning: GMM_BATCH_SHAPE, then
// GMM_BATCH_CULL=1 (first culled shape), else the label shape.
int batch_default_spec(int kmax) {
  const char *e = getenv("GMM_BATCH_SHAPE");
  if (e && *e) {
    const int s = batch_spec_by_name(e);
    if (s >= 0) return s;
  }
  const char *off = getenv("GMM_CULL");
  const char *on = getenv("GMM_BATCH_CULL");
  if (on && on[0] == '1' && !(off && off[0] == '0')) return 2;
  return kmax <= 512 ? 0 : 1;
}

// ---- batched autotuner: per (device, B, K_max, log2 sum N_f K_f)
struct BatchTune {
  int dev, B, kmax, bucket, spec;
};
std::mutex g_btune_mu;
std::vector<BatchTune> g_btune;
bool g_btune_loaded = false;

int evals_bucket(int64_t e) {
  int b = 0;
  while (e > 1) { e >>= 1; ++b; }
  return b;
}

void btune_load_locked() {
  if (g_btune_loaded) return;
  g_btune_loaded = true;
  const char *path = getenv("GMM_AUTOTUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char tag[16], name[64];
  int B, kmax, bucket;
  while (fscanf(f, "%15s", tag) == 1) {
    if (strcmp(tag, "batch") == 0 && fscanf(f, "%d %d %d %63s", &B, &kmax, &bucket, name) == 4) {
      const int s = batch_spec_by_name(name);
      if (s >= 0) g_btune.push_back(BatchTune{-1, B, kmax, bucket, s});
    } else {
      int c;
      while ((c = fgetc(f)) != EOF && c != '\n') {}
    }
  }
  fclose(f);
}

int btune_lookup(const BatchPlan &bp) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_btune_mu);
  btune_load_locked();
  const int bucket = evals_bucket(bp.evals);
  for (const auto &t : g_btune)
    if ((t.dev == dev || t.dev == -1) && t.B == bp.B && t.kmax == bp.Kmax && t.bucket == bucket)
      return t.spec;
  return -1;
}

void btune_store(const BatchPlan &bp, int spec) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_btune_mu);
  const int bucket = evals_bucket(bp.evals);
  g_btune.push_back(BatchTune{dev, bp.B, bp.Kmax, bucket, spec});
  const char *path = getenv("GMM_AUTOTUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "batch %d %d %d %s\n", bp.B, bp.Kmax, bucket, kBatchSpec[spec].name);
  fclose(f);
}

// Every frame of the staged batch in its own Morton order: raw4 -> pts4.
gmm_status batch_spatial_order(const BatchPlan &bp, void *ws, hipStream_t s) {
  const int64_t np = bp.tiles * kBatchT;
  const int nblk = bp.sort_blocks;
  const BFrame *frames = reinterpret_cast<const BFrame *>(at<unsigned char>(ws, bp.plan));
  hipLaunchKernelGGL(frame_box_kernel, dim3(bp.B), dim3(kSortThreads), 0, s,
                     at<float4>(ws, bp.raw4), frames, kBatchT, at<float>(ws, bp.box6));
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(morton_frames_kernel, dim3(64, bp.B), dim3(kSortThreads), 0, s,
                     at<float4>(ws, bp.raw4), frames, kBatchT, kBatchCullT,
                     at<float>(ws, bp.box6), at<unsigned>(ws, bp.keys[0]),
                     at<unsigned>(ws, bp.vals[0]));
  HIP_TRY(hipGetLastError());
  int src = 0;
  for (int shift = 0; shift < 32; shift += 8, src = 1 - src) {
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nblk), dim3(kSortThreads), 0, s,
                       at<unsigned>(ws, bp.keys[src]), np, shift,
                       at<unsigned>(ws, bp.hist), nblk);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(radix_scan_kernel, dim3(256), dim3(kSortThreads), 0, s,
                       at<unsigned>(ws, bp.hist), nblk, at<unsigned>(ws, bp.dtot));
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblk), dim3(kSortThreads), 0, s,
                       at<unsigned>(ws, bp.keys[src]), at<unsigned>(ws, bp.vals[src]),
                       np, shift, at<unsigned>(ws, bp.hist), nblk,
                       at<unsigned>(ws, bp.dtot), at<unsigned>(ws, bp.keys[1 - src]),
                       at<unsigned>(ws, bp.vals[1 - src]));
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((np + kSortThreads - 1) / kSortThreads)),
                     dim3(kSortThreads), 0, s, at<float4>(ws, bp.raw4),
                     at<unsigned>(ws, bp.vals[src]), np, at<float4>(ws, bp.pts4));
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

struct BatchRun {
  const BatchPlan *bp = nullptr;
  void *ws = nullptr;
  hipStream_t s = nullptr;
  int cur = 0;
  bool timed = false;   // profiling: time the soft passes' tile launches
};

// The tile launch of one pass with shape variant v.
void batch_tiles(BatchRun &r, const BatchVariant &v, int mode) {
  const BatchPlan &bp = *r.bp;
  for (const auto &c : v.sets)
    c.launch(c, r.s, at<float4>(r.ws, bp.pts4), bp.sort ? at<float4>(r.ws, bp.tsph) : nullptr,
             at<float>(r.ws, bp.cpar[r.cur]), at<float4>(r.ws, bp.shift[r.cur]),
             at<double>(r.ws, bp.part), at<unsigned char>(r.ws, bp.plan), v.frames_off, mode);
}

gmm_status batch_pass(BatchRun &r, int mode, int umode, double reg,
                      double *loglik, int ll_stride, int ll_index,
                      float *out_w = nullptr, float *out_mu = nullptr,
                      float *out_cov = nullptr) {
  const BatchPlan &bp = *r.bp;
  unsigned char *plan = at<unsigned char>(r.ws, bp.plan);
  const BatchVariant &v = bp.vars[mode == kLabels ? bp.lab_var : bp.soft_var];
  const BFrame *frames = reinterpret_cast<const BFrame *>(plan + v.frames_off);
  const bool timed = r.timed && mode == kSoftStats;
  EventPair pp;
  if (timed) {
    if (!make_pair(&pp)) return fail(GMM_ERR_DEVICE, "profiling event allocation failed");
    pp.reps = g_prof.reps;
    g_prof.pending.push_back(pp);
    int64_t pairs = 0;
    for (const auto &F : v.frames)
      pairs += (int64_t)((F.n + kBatchT - 1) / kBatchT) * F.K;
    g_prof.pairs_all += pairs * g_prof.reps;
    g_prof.pairs_dense += pairs * g_prof.reps;
    HIP_TRY(hipEventRecord(pp.a, r.s));
  }
  for (int rep = 0; rep < (timed ? g_prof.reps : 1); ++rep) {
    batch_tiles(r, v, mode);
    HIP_TRY(hipGetLastError());
  }
  if (timed) HIP_TRY(hipEventRecord(pp.b, r.s));
  const int only_L = mode == kSoftLogLik;
  const int ncx = (only_L ? 1 : (bp.ncols_max + 63) / 64);
  hipLaunchKernelGGL(reduce_frames_kernel, dim3(bp.B, ncx), dim3(256), 0, r.s,
                     at<double>(r.ws, bp.part), frames, only_L,
                     at<double>(r.ws, bp.red));
  HIP_TRY(hipGetLastError());
  const int nxt = 1 - r.cur;
  const size_t lds = ((size_t)bp.ncols_max + kUpdThreads + 2 * (size_t)bp.Kmax) * sizeof(double);
  hipLaunchKernelGGL(update_frames_kernel, dim3(bp.B), dim3(kUpdThreads), lds,
                     r.s, at<double>(r.ws, bp.red), frames, mode, umode, reg,
                     at<float>(r.ws, bp.cpar[r.cur]), at<float4>(r.ws, bp.shift[r.cur]),
                     at<float>(r.ws, bp.cpar[nxt]), at<float4>(r.ws, bp.shift[nxt]),
                     at<double>(r.ws, bp.th64), loglik, ll_stride, ll_index,
                     out_w, out_mu, out_cov, at<uint32_t>(r.ws, bp.status));
  HIP_TRY(hipGetLastError());
  if (umode != kUpdNone) r.cur = nxt;
  return GMM_OK;
}

// theta_0: the one-hot M-step of the labels, or the caller's parameters.
gmm_status batch_start(BatchRun &r, const int32_t *labels, const float *w, const float *mu,
                       const float *cov, double reg) {
  const BatchPlan &bp = *r.bp;
  gmm_status st;
  if (labels) {
    if ((st = batch_pass(r, kLabels, kUpdMeanOnly, reg, nullptr, 1, 0)) != GMM_OK) return st;
    return batch_pass(r, kLabels, kUpdFull, reg, nullptr, 1, 0);
  }
  const BFrame *frames = reinterpret_cast<const BFrame *>(at<unsigned char>(r.ws, bp.plan));
  hipLaunchKernelGGL(precompute_frames_kernel, dim3(bp.B), dim3(kPreThreads), 0,
                     r.s, w, mu, cov, frames, at<float>(r.ws, bp.cpar[r.cur]),
                     at<float4>(r.ws, bp.shift[r.cur]), at<double>(r.ws, bp.th64),
                     at<uint32_t>(r.ws, bp.status));
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

gmm_status enqueue_batched(BatchRun &r, const int32_t *labels, float *w,
                           float *mu, float *cov, double *loglik,
                           const gmm_fit_opts *opts) {
  gmm_status st;
  const int T = opts->iters, ll = T + 1;
  const double reg = opts->reg_covar;
  if ((st = batch_start(r, labels, w, mu, cov, reg)) != GMM_OK) return st;
  for (int t = 0; t < T; ++t) {
    if (opts->moment_mode == GMM_MOMENTS_TWO_PASS) {
      if ((st = batch_pass(r, kSoftStats, kUpdMeanOnly, reg, loglik, ll, t)) != GMM_OK) return st;
      if ((st = batch_pass(r, kSoftStats, kUpdFull, reg, nullptr, ll, t)) != GMM_OK) return st;
    } else {
      if ((st = batch_pass(r, kSoftStats, kUpdFull, reg, loglik, ll, t)) != GMM_OK) return st;
    }
  }
  return batch_pass(r, kSoftLogLik, kUpdNone, reg, loglik, ll, T, w, mu, cov);
}

// Autotuning: from theta_0 (which no tile pass changes), one soft pass of
// every shape in the plan, timed over 3 launches after a warm-up; the
// fastest becomes the soft shape.
gmm_status batch_autotune(BatchRun &r, BatchPlan &bp) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best = -1;
  float best_ms = 0.0f;
  for (int i = 0; i < (int)bp.vars.size(); ++i) {
    const BatchVariant &v = bp.vars[i];
    batch_tiles(r, v, kSoftStats);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(e0, r.s));
    for (int rep = 0; rep < 3; ++rep) batch_tiles(r, v, kSoftStats);
    HIP_TRY(hipEventRecord(e1, r.s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (best < 0 || ms < best_ms) {
      best = i;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  bp.soft_var = best;
  btune_store(bp, bp.vars[best].spec);
  return GMM_OK;
}


// The soft shape of a call: forced by GMM_BATCH_SHAPE, else the tuned one
// (autotuning on), else the default; -2 when autotuning is on and this
// batch has no tuned shape yet.
int batch_soft_spec(const BatchPlan &bp) {
  const char *e = getenv("GMM_BATCH_SHAPE");
  if (e && *e && batch_spec_by_name(e) >= 0) return batch_spec_by_name(e);
  if (autotune_on()) {
    const int s = btune_lookup(bp);
    return s >= 0 ? s : -2;
  }
  return batch_default_spec(bp.Kmax);
}

// Index of spec in the plan's shapes (the label shape when it is absent).
int batch_var_index(const BatchPlan &bp, int spec) {
  for (int i = 0; i < (int)bp.vars.size(); ++i)
    if (bp.vars[i].spec == spec) return i;
  return bp.lab_var;
}

}  // namespace

// ------------------------------------------------------ allocation-free fit
// Device memory of gmm_fit_noalloc: one array per GPU, in the code object,
// held until the process ends.  Host code never passes the symbol itself to
// a kernel (on the host it names a stand-in, not device memory): the device
// address is read once per device with hipGetSymbolAddress and kept.
static __device__ __align__(256) unsigned char scratch[GMM_FIT_NOALLOC_MAX_BYTES];

namespace {

static_assert(GMM_FIT_NOALLOC_MAX_BYTES % 256 == 0, "scratch size");
constexpr size_t kScratchBytes = GMM_FIT_NOALLOC_MAX_BYTES;
std::mutex g_scratch_mu;
void *g_scratch_dev[64];

gmm_status scratch_address(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(GMM_ERR_DEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255))
      return fail(GMM_ERR_DEVICE, "scratch array address %p unusable", p);
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
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
  return ws_layout(n, k, c, 0, 0, true).total;
}

gmm_status gmm_fit(const float *pts, int64_t n, int32_t k,
                   const int32_t *init_labels, float *w, float *mu, float *cov,
                   double *loglik, const gmm_fit_opts *opts, void *ws,
                   size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  Run r;
  gmm_status st = fit_setup(pts, n, k, w, mu, cov, opts, stream, &r);
  if (st != GMM_OK) return st;
  WsGuard guard;
  if ((st = get_ws(&ws, &ws_bytes, r.L.total, r.s, &guard)) != GMM_OK) return st;
  r.ws = ws;
  const bool sync = !(opts->flags & GMM_FLAG_ASYNC);

  // Profiled calls launch directly: the HIP runtime does not time events
  // that a captured graph records.
  if (graphs_enabled() && !guard.ptr && g_prof.reps == 0) {
    FitKey key{pts, init_labels, w, mu, cov, loglik, ws, n, ws_bytes,
               opts->reg_covar, opts->tol, k, opts->iters, opts->moment_mode, 0,
               reinterpret_cast<const void *>(r.c.launch),
               r.cull ? reinterpret_cast<const void *>(r.cc.launch) : nullptr,
               sort_enabled(), r.fused, r.small, small_give_up()};
    (void)hipGetDevice(&key.dev);
    std::lock_guard<std::mutex> lk(g_graph_mu);
    bool found = false;
    GraphEntry *e = graph_slot(key, &found);
    if (found && !e->exec) {
      // second call with these arguments: capture the whole fit
      hipStream_t cs = capture_stream();
      if (cs && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        Run rc = r;
        rc.s = cs;
        gmm_status cst = enqueue_fit(rc, pts, n, init_labels, w, mu, cov, loglik, opts, false);
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
      return finish(r, sync);
    }
  }
  r.sink = g_prof.reps > 0 ? &g_prof.pending : nullptr;
  if ((st = enqueue_fit(r, pts, n, init_labels, w, mu, cov, loglik, opts, true)) != GMM_OK) return st;
  return finish(r, sync);
}

gmm_status gmm_fit_noalloc(const float *pts, int64_t n, int32_t k,
                           const int32_t *init_labels, float *w, float *mu,
                           float *cov, double *loglik, const gmm_fit_opts *opts,
                           void *stream) {
  g_err[0] = 0;
  Run r;
  gmm_status st = fit_setup(pts, n, k, w, mu, cov, opts, stream, &r);
  if (st != GMM_OK) return st;
  if (opts->flags & GMM_FLAG_ASYNC)
    return fail(GMM_ERR_INVALID_ARG, "gmm_fit_noalloc always synchronises (no GMM_FLAG_ASYNC)");
  if (r.L.total > kScratchBytes)
    return fail(GMM_ERR_UNSUPPORTED,
                "a fit of n=%lld k=%d needs %zu bytes of scratch; the allocation-free fit holds %zu",
                (long long)n, k, r.L.total, kScratchBytes);
  if ((st = scratch_address(&r.ws)) != GMM_OK) return st;
  // direct launches only: no graph capture, no autotuning and no profiling
  // events, each of which allocates
  r.sink = nullptr;
  if ((st = enqueue_fit(r, pts, n, init_labels, w, mu, cov, loglik, opts, false)) != GMM_OK)
    return st;
  return finish(r, true);
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
  Run r;
  r.K = k;
  if (!pick_cfg(k, n, &r.c)) return fail(GMM_ERR_UNSUPPORTED, "no launch configuration for k=%d", k);
  r.cull = pick_cull_cfg(k, n, &r.cc);
  r.L = ws_layout(n, k, r.c);
  r.s = static_cast<hipStream_t>(stream);
  WsGuard guard;
  if ((st = get_ws(&ws, &ws_bytes, r.L.total, r.s, &guard)) != GMM_OK) return st;
  r.ws = ws;
  if ((st = run_init(r, false)) != GMM_OK) return st;
  const float *Rt = nullptr;
  if (pose6) {
    hipLaunchKernelGGL(pose_kernel, dim3(1), dim3(64), 0, r.s, pose6,
                       at<double>(ws, r.L.pose64), at<float>(ws, r.L.rt32));
    HIP_TRY(hipGetLastError());
    Rt = at<float>(ws, r.L.rt32);
  }
  if ((st = stage(r, pts, n, nullptr, Rt)) != GMM_OK) return st;
  if ((st = run_precompute(r, w, mu, cov)) != GMM_OK) return st;
  if (g_prof.reps > 0) {
    r.sink = &g_prof.pending;
    r.time_loglik = true;
  }
  return run_pass(r, kSoftLogLik, kUpdNone, 0.0, out_L, out_lse);
}


size_t gmm_fit_batched_workspace_size(int32_t B, const int64_t *pt_off,
                                      const int32_t *k_off,
                                      const gmm_fit_opts *opts) {
  (void)opts;
  g_err[0] = 0;
  if (!pt_off || !k_off || B <= 0 || pt_off[0] != 0 || k_off[0] != 0) return 0;
  // sized for every launch shape the call may tune to or be forced to
  BatchPlan bp;
  if (make_batch_plan(B, pt_off, k_off, &bp, true) != GMM_OK) return 0;
  return bp.total;
}

const char *gmm_fit_batched_config(int32_t B, const int64_t *pt_off, const int32_t *k_off) {
  g_err[0] = 0;
  if (!pt_off || !k_off || B <= 0 || pt_off[0] != 0 || k_off[0] != 0) return "";
  BatchPlan bp;
  if (make_batch_plan(B, pt_off, k_off, &bp, false) != GMM_OK) return "";
  const int s = batch_soft_spec(bp);
  if (s < 0) return "";
  // a shape that cannot run these frames falls back to the label shape
  if (make_batch_plan(B, pt_off, k_off, &bp, false, s) != GMM_OK) return "";
  return kBatchSpec[bp.vars[batch_var_index(bp, s)].spec].name;
}

gmm_status gmm_fit_batched(int32_t B, const float *pts, const int64_t *pt_off,
                           const int32_t *k_off, const int32_t *init_labels,
                           float *w, float *mu, float *cov, double *loglik,
                           const gmm_fit_opts *opts, void *ws, size_t ws_bytes,
                           void *stream) {
  g_err[0] = 0;
  if (!pts || !pt_off || !k_off || !w || !mu || !cov || !opts)
    return fail(GMM_ERR_INVALID_ARG, "NULL pointer argument");
  if (opts->iters < 0) return fail(GMM_ERR_INVALID_ARG, "iters < 0");
  if (!(opts->reg_covar >= 0.0) || !isfinite(opts->reg_covar))
    return fail(GMM_ERR_INVALID_ARG, "reg_covar must be finite and >= 0");
  if (opts->moment_mode != GMM_MOMENTS_SHIFTED &&
      opts->moment_mode != GMM_MOMENTS_TWO_PASS)
    return fail(GMM_ERR_INVALID_ARG, "unknown moment_mode");
  if (opts->flags & ~(GMM_FLAG_ASYNC | GMM_FLAG_DETERMINISTIC))
    return fail(GMM_ERR_INVALID_ARG, "unknown flags");
  if (opts->tol != 0.0) return fail(GMM_ERR_INVALID_ARG, "batched fits run a fixed T (tol = 0)");
  if (B <= 0) return fail(GMM_ERR_INVALID_ARG, "B=%d must be positive", B);
  if (pt_off[0] != 0 || k_off[0] != 0)
    return fail(GMM_ERR_INVALID_ARG, "offsets must start at 0");
  // the plan: every shape when tuning now, else the label shape and the soft shape
  BatchPlan bp;
  gmm_status st = make_batch_plan(B, pt_off, k_off, &bp, false);
  if (st != GMM_OK) return st;
  int spec = batch_soft_spec(bp);
  const bool tune = spec == -2;
  if ((st = make_batch_plan(B, pt_off, k_off, &bp, tune, tune ? -1 : spec)) != GMM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  WsGuard guard;
  if ((st = get_ws(&ws, &ws_bytes, bp.total, s, &guard)) != GMM_OK) return st;
  // plan upload (the host buffer lives until the copy has completed), status
  // and shift reset, staging of every frame into its tiles (padded to
  // kBatchCullT points), per-frame Morton order and tile spheres when the
  // plan has a culled shape
  auto prepare = [&]() -> gmm_status {
    std::vector<unsigned char> host(bp.plan_bytes, 0);
    memcpy(host.data(), bp.base.data(), sizeof(BFrame) * B);
    for (const auto &v : bp.vars) {
      memcpy(host.data() + v.frames_off, v.frames.data(), sizeof(BFrame) * B);
      for (const auto &c : v.sets) {
        memcpy(host.data() + c.seg_off, c.segs.data(), sizeof(BSeg) * c.segs.size());
        memcpy(host.data() + c.blk_off, c.blk.data(), sizeof(int) * c.blk.size());
      }
    }
    HIP_TRY(hipMemcpyAsync(at<unsigned char>(ws, bp.plan), host.data(),
                           bp.plan_bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    hipLaunchKernelGGL(init_kernel, dim3(64), dim3(256), 0, s,
                       at<uint32_t>(ws, bp.status), nullptr, 0,
                       init_labels ? at<float4>(ws, bp.shift[0]) : nullptr, bp.Ktot);
    HIP_TRY(hipGetLastError());
    const size_t stage_to = bp.sort ? bp.raw4 : bp.pts4;
    for (int f = 0; f < B; ++f) {
      const int64_t n = pt_off[f + 1] - pt_off[f];
      const int64_t npad = ((n + kBatchCullT - 1) / kBatchCullT) * kBatchCullT;
      hipLaunchKernelGGL(stage_kernel, dim3((unsigned)((npad + 255) / 256)), dim3(256),
                         0, s, pts + 3 * pt_off[f], n, npad,
                         init_labels ? init_labels + pt_off[f] : nullptr,
                         bp.base[f].K, nullptr,
                         at<float4>(ws, stage_to) + bp.base[f].toff * kBatchT,
                         at<uint32_t>(ws, bp.status));
      HIP_TRY(hipGetLastError());
    }
    if (bp.sort) {
      gmm_status so = batch_spatial_order(bp, ws, s);
      if (so != GMM_OK) return so;
      const int64_t nt = bp.tiles * kBatchT / kBatchCullT;
      hipLaunchKernelGGL(tile_sphere_kernel, dim3((unsigned)nt), dim3(256), 0, s,
                         at<float4>(ws, bp.pts4), kBatchCullT, at<float4>(ws, bp.tsph));
      HIP_TRY(hipGetLastError());
    }
    return GMM_OK;
  };
  if ((st = prepare()) != GMM_OK) return st;
  BatchRun r;
  r.ws = ws;
  r.s = s;
  if (tune) {
    // theta_0 and a few EM iterations with the label shape (the components
    // of a k-means start are more compact than they stay, which favours
    // culling), one timed soft pass per shape; then the plan of the winner
    // alone, staged afresh, so that the fit equals one forced to that shape
    r.bp = &bp;
    if ((st = batch_start(r, init_labels, w, mu, cov, opts->reg_covar)) != GMM_OK) return st;
    bp.soft_var = bp.lab_var;
    for (int t = 0; t < std::min(opts->iters, kBatchTuneIters); ++t)
      if ((st = batch_pass(r, kSoftStats, kUpdFull, opts->reg_covar, nullptr, 1, 0)) != GMM_OK)
        return st;
    if ((st = batch_autotune(r, bp)) != GMM_OK) return st;
    spec = bp.vars[bp.soft_var].spec;
    if ((st = make_batch_plan(B, pt_off, k_off, &bp, false, spec)) != GMM_OK) return st;
    if ((st = prepare()) != GMM_OK) return st;
    r.cur = 0;
  }
  bp.soft_var = batch_var_index(bp, spec);
  r.bp = &bp;
  debug_cfg("fit_batched", bp.Kmax, bp.tiles * kBatchT, kBatchSpec[bp.vars[bp.soft_var].spec].name,
            (int)bp.vars[bp.soft_var].sets.size(), kBatchSpec[bp.vars[bp.soft_var].spec].block,
            bp.vars[bp.soft_var].sets[0].lds);
  // the iteration loop as one graph (direct launches when capture fails or
  // when the tile kernels are being timed)
  r.timed = g_prof.reps > 0;
  bool done = false;
  if (graphs_enabled() && !r.timed) {
    hipStream_t cs = capture_stream();
    hipEvent_t ev = nullptr;
    if (cs && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
        hipEventRecord(ev, s) == hipSuccess && hipStreamWaitEvent(cs, ev, 0) == hipSuccess &&
        hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      BatchRun rc = r;
      rc.s = cs;
      gmm_status cst = enqueue_batched(rc, init_labels, w, mu, cov, loglik, opts);
      hipGraph_t g = nullptr;
      hipError_t ee = hipStreamEndCapture(cs, &g);
      hipGraphExec_t exec = nullptr;
      if (cst == GMM_OK && ee == hipSuccess && g &&
          hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess) {
        hipError_t le = hipGraphLaunch(exec, s);
        done = le == hipSuccess;
        if (done) HIP_TRY(hipStreamSynchronize(s));
        (void)hipGraphExecDestroy(exec);
      }
      if (g) (void)hipGraphDestroy(g);
    }
    if (ev) (void)hipEventDestroy(ev);
    (void)hipGetLastError();
  }
  if (!done && (st = enqueue_batched(r, init_labels, w, mu, cov, loglik, opts)) != GMM_OK)
    return st;
  if (opts->flags & GMM_FLAG_ASYNC) return GMM_OK;
  uint32_t bits = 0;
  HIP_TRY(hipMemcpyAsync(&bits, at<uint32_t>(ws, bp.status), sizeof bits,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return status_from_bits(bits);
}

// ------------------------------------------------------- k-means++ seeding

struct KppLayout {
  size_t status, D, T, D2, T2, total;
  int64_t nch;
  bool fused;   // one launch per round (double-buffered D, T)
};

KppLayout kpp_layout(int64_t n) {
  KppLayout L;
  L.nch = (n + kKppChunk - 1) / kKppChunk;
  size_t o = 0;
  L.status = o; o = align256(o + sizeof(uint32_t));
  L.D = o; o = align256(o + (size_t)n * sizeof(double));
  L.T = o; o = align256(o + (size_t)L.nch * sizeof(double));
  L.fused = L.nch <= kKppFuseChunks;
  L.D2 = L.T2 = 0;
  if (L.fused) {
    L.D2 = o; o = align256(o + (size_t)n * sizeof(double));
    L.T2 = o; o = align256(o + (size_t)L.nch * sizeof(double));
  }
  L.total = o;
  return L;
}

size_t gmm_kmeanspp_workspace_size(int64_t n, int32_t k) {
  g_err[0] = 0;
  if (check_sizes(n, k, true) != GMM_OK) return 0;
  return kpp_layout(n).total;
}

gmm_status gmm_kmeanspp(const float *pts, int64_t n, int32_t k, const double *u,
                        int64_t *centres, int32_t *labels, void *ws, size_t ws_bytes,
                        void *stream) {
  g_err[0] = 0;
  gmm_status st = check_sizes(n, k, true);
  if (st != GMM_OK) return st;
  if (!pts || !u || !centres) return fail(GMM_ERR_INVALID_ARG, "NULL pointer argument");
  const KppLayout L = kpp_layout(n);
  hipStream_t s = static_cast<hipStream_t>(stream);
  WsGuard guard;
  if ((st = get_ws(&ws, &ws_bytes, L.total, s, &guard)) != GMM_OK) return st;
  uint32_t *status = at<uint32_t>(ws, L.status);
  double *D = at<double>(ws, L.D), *T = at<double>(ws, L.T);
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(256), 0, s, status, nullptr, 0,
                     nullptr, 0);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(kpp_first_kernel, dim3(1), dim3(256), 0, s, u, k, n, centres,
                     status);
  HIP_TRY(hipGetLastError());
  const dim3 ugrid((unsigned)((L.nch + kKppUpdChunks - 1) / kKppUpdChunks));
  if (L.fused && k >= 2) {
    // round j: centre j from buffer (j - 1) & 1, distances into buffer j & 1
    double *Db[2] = {D, at<double>(ws, L.D2)}, *Tb[2] = {T, at<double>(ws, L.T2)};
    hipLaunchKernelGGL(kpp_update_kernel, ugrid, dim3(kKppUpdThreads), 0, s, pts, n, centres, 0,
                       Db[0], Tb[0], L.nch, status);
    HIP_TRY(hipGetLastError());
    for (int j = 1; j + 1 < k; ++j) {
      hipLaunchKernelGGL(kpp_round_kernel, ugrid, dim3(kKppUpdThreads), 0, s, pts, n, u, j,
                         centres, Db[(j - 1) & 1], Tb[(j - 1) & 1], Db[j & 1], Tb[j & 1], L.nch);
      HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(kpp_select_kernel, dim3(1), dim3(kKppSelThreads), 0, s, Db[k & 1],
                       Tb[k & 1], n, u, k - 1, centres);
    HIP_TRY(hipGetLastError());
  } else {
    for (int j = 1; j < k; ++j) {
      hipLaunchKernelGGL(kpp_update_kernel, ugrid, dim3(kKppUpdThreads), 0, s, pts, n, centres,
                         j - 1, D, T, L.nch, status);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(kpp_select_kernel, dim3(1), dim3(kKppSelThreads), 0, s, D, T, n, u, j,
                         centres);
      HIP_TRY(hipGetLastError());
    }
  }
  if (!labels && k == 1) {  // no distances formed: check the points alone
    hipLaunchKernelGGL(kpp_check_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       pts, n, status);
    HIP_TRY(hipGetLastError());
  }
  if (labels) {
    hipLaunchKernelGGL(kpp_label_kernel,
                       dim3((unsigned)((n + kKppLabelThreads - 1) / kKppLabelThreads)),
                       dim3(kKppLabelThreads), (size_t)k * 3 * sizeof(double), s, pts, n,
                       centres, k, labels, status);
    HIP_TRY(hipGetLastError());
  }
  uint32_t bits = 0;
  HIP_TRY(hipMemcpyAsync(&bits, status, sizeof bits, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return status_from_bits(bits);
}

gmm_status gmm_set_autotune(int on) {
  g_autotune = on ? 1 : 0;
  return GMM_OK;
}

const char *gmm_tile_config(int64_t n, int32_t k) {
  g_err[0] = 0;
  if (check_sizes(n, k, false) != GMM_OK) return "";
  TileCfg c;
  CullCfg cc;
  if (pick_cull_cfg(k, n, &cc)) return cc.name;
  const int f = forced_candidate();
  if (f >= 0 && kCand[f](k, n, &c)) return kCandName[f];
  const int t = tuned_candidate(k, n);
  if (t >= 0 && kCand[t](k, n, &c)) return kCandName[t];
  const int d = default_candidate(k, n);
  return d >= 0 ? kCandName[d] : "";
}

gmm_status gmm_profile_enable(int reps) {
  g_err[0] = 0;
  if (reps < 0 || reps > 64)
    return fail(GMM_ERR_INVALID_ARG, "profile repeats must be in [0, 64] (got %d)", reps);
  if (reps > 0) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (!g_prof.dpairs || g_prof.dpairs_dev != dev) {
      unsigned long long *p = nullptr;
      HIP_TRY(hipMalloc(&p, sizeof(unsigned long long)));
      HIP_TRY(hipMemset(p, 0, sizeof(unsigned long long)));
      g_prof.dpairs = p;  // one counter per thread and device, kept
      g_prof.dpairs_dev = dev;
    }
  }
  g_prof.reps = reps;
  return GMM_OK;
}

gmm_status gmm_profile_pairs(int64_t *evaluated, int64_t *all) {
  g_err[0] = 0;
  unsigned long long dev_pairs = 0;
  if (g_prof.dpairs) {
    HIP_TRY(hipMemcpy(&dev_pairs, g_prof.dpairs, sizeof dev_pairs, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(g_prof.dpairs, 0, sizeof(unsigned long long)));
  }
  if (evaluated) *evaluated = g_prof.pairs_dense + (int64_t)dev_pairs;
  if (all) *all = g_prof.pairs_all;
  g_prof.pairs_dense = 0;
  g_prof.pairs_all = 0;
  return GMM_OK;
}

gmm_status gmm_profile_read(double *tile_ms_total, int64_t *tile_launches) {
  hipError_t e = add_elapsed(g_prof.pending);
  destroy_pairs(g_prof.pending);
  if (e != hipSuccess) return fail(GMM_ERR_DEVICE, "profiling: %s", hipGetErrorString(e));
  if (tile_ms_total) *tile_ms_total = g_prof.ms_total;
  if (tile_launches) *tile_launches = g_prof.launches;
  g_prof.ms_total = 0.0;
  g_prof.launches = 0;
  return GMM_OK;
}

size_t gmm_loglik_backward_workspace_size(int64_t n, int32_t k) {
  g_err[0] = 0;
  if (check_sizes(n, k, false) != GMM_OK) return 0;
  TileCfg c;
  BwdCfg bc;
  if (!pick_cfg(k, n, &c) || !pick_bwd_cfg(k, n, &bc)) return 0;
  return ws_layout(n, k, c, kBwdExtra, bc.grid).total;
}

gmm_status gmm_loglik_backward(const float *pts, int64_t n, const float *pose6,
                               int32_t k, const float *w, const float *mu,
                               const float *cov, const double *grad_L,
                               float *g_pose6, float *g_pts, float *g_w,
                               float *g_mu, float *g_cov, void *ws,
                               size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  gmm_status st = check_sizes(n, k, false);
  if (st != GMM_OK) return st;
  if (!pts || !w || !mu || !cov)
    return fail(GMM_ERR_INVALID_ARG, "NULL pointer argument");
  Run r;
  r.K = k;
  BwdCfg bc;
  if (!pick_cfg(k, n, &r.c) || !pick_bwd_cfg(k, n, &bc))
    return fail(GMM_ERR_UNSUPPORTED, "no backward configuration for k=%d", k);
  r.L = ws_layout(n, k, r.c, kBwdExtra, bc.grid);
  r.s = static_cast<hipStream_t>(stream);
  WsGuard guard;
  if ((st = get_ws(&ws, &ws_bytes, r.L.total, r.s, &guard)) != GMM_OK) return st;
  r.ws = ws;
  if ((st = run_init(r, false)) != GMM_OK) return st;
  const float *Rt = nullptr;
  const double *pose64 = nullptr;
  if (pose6) {
    hipLaunchKernelGGL(pose_kernel, dim3(1), dim3(64), 0, r.s, pose6,
                       at<double>(ws, r.L.pose64), at<float>(ws, r.L.rt32));
    HIP_TRY(hipGetLastError());
    Rt = at<float>(ws, r.L.rt32);
    pose64 = at<double>(ws, r.L.pose64);
  }
  if ((st = stage(r, pts, n, nullptr, Rt)) != GMM_OK) return st;
  if ((st = run_precompute(r, w, mu, cov)) != GMM_OK) return st;
  // the backward kernel has its own tile size (the forward's shape, which a
  // forced or tuned configuration may set to 128 points, does not apply)
  TileArgs a;
  a.ntiles = (int)(r.L.npad / bc.tile);
  a.K = k;
  a.KC = k;
  a.P = bc.P;
  a.mode = kSoftStats;
  a.ncols = r.L.ncols;
  // profiling: the backward tile kernel is timed like the fit's E+M passes
  // (it overwrites its per-point outputs and partial rows, so repeats
  // change nothing)
  EventPair pp;
  const bool timed = g_prof.reps > 0;
  if (timed) {
    if (!make_pair(&pp)) return fail(GMM_ERR_DEVICE, "profiling event allocation failed");
    pp.reps = g_prof.reps;
    g_prof.pending.push_back(pp);
    const int64_t all = (int64_t)g_prof.reps * a.ntiles * k;
    g_prof.pairs_all += all;
    g_prof.pairs_dense += all;
    HIP_TRY(hipEventRecord(pp.a, r.s));
  }
  for (int rep = 0; rep < (timed ? g_prof.reps : 1); ++rep) {
    bc.launch(bc, r.s, at<float4>(ws, r.L.pts4), at<float>(ws, r.L.cpar[r.cur]),
              at<float4>(ws, r.L.shift[r.cur]), Rt, grad_L,
              at<double>(ws, r.L.part), g_pts, a, n);
    HIP_TRY(hipGetLastError());
  }
  if (timed) HIP_TRY(hipEventRecord(pp.b, r.s));
  const int ncx = (r.L.ncols + 63) / 64;
  hipLaunchKernelGGL(reduce_rows_kernel<256>, dim3(ncx, kRedChunks), dim3(256), 0,
                     r.s, at<double>(ws, r.L.part), bc.grid, r.L.ncols, 0,
                     at<double>(ws, r.L.red));
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(bwd_finish_kernel, dim3(1), dim3(256), 0, r.s,
                     at<double>(ws, r.L.red), r.L.ncols, k, w, cov, pose64,
                     grad_L, g_pose6, g_w, g_mu, g_cov,
                     at<uint32_t>(ws, r.L.status));
  HIP_TRY(hipGetLastError());
  return GMM_OK;
}

}  // extern "C"
