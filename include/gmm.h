/*
 * gmm.h - C ABI of the MI355X (gfx950) Gaussian-mixture EM library.
 *
 * The library fits 3D Gaussian mixture models to point clouds by
 * expectation-maximization and evaluates / differentiates the mixture
 * log-likelihood of a rigidly transformed cloud.  The method is the EM of
 * Goel, Tabib et al., "GIRA" (arXiv 2307.00071), Sec. V "Expectation
 * Maximization": the E-step computes responsibilities (eq. 1) in the log
 * domain (eq. 2) from the Cholesky-precision form of the Gaussian
 * log-density (eq. 3); the M-step (named, not written out, in that
 * section) is the standard maximum-likelihood update of weights, means and
 * full covariances, here with a diagonal regulariser lambda.
 *
 * Conventions shared by every entry point
 *  - Device pointers unless stated otherwise; every buffer is owned by the
 *    caller.  The library keeps no per-call state besides the caller's
 *    workspace, so calls with distinct workspaces are re-entrant.
 *  - Points: float32, row-major N x 3 (x, y, z), no alignment requirement
 *    beyond 4 bytes.
 *  - Mixture: weights w[K] (float32, > 0), means mu[K][3], covariances
 *    cov[K][3][3] (row-major; the LOWER triangle is read, a symmetric
 *    matrix is written).
 *  - All work is enqueued on `stream` (a hipStream_t; NULL = the legacy
 *    default stream).  Host-side argument errors return before anything is
 *    enqueued.  Device-side conditions (a covariance that is not SPD, a
 *    non-finite point or result, a label out of range) are collected in a
 *    status word inside the workspace; entry points that synchronise
 *    return it, the others leave it for gmm_workspace_status().
 *  - Workspace: `ws` is a device buffer of at least the size reported by
 *    the matching *_workspace_size() call, aligned to 256 bytes.  With
 *    ws == NULL the library allocates one stream-ordered (hipMallocAsync)
 *    and frees it after the call.
 *  - Limits: 1 <= K <= GMM_MAX_K, 1 <= N <= GMM_MAX_N, K <= N for fits.
 */
#ifndef GMM_MI355X_H
#define GMM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GMM_MAX_K 1024
#define GMM_MAX_N ((int64_t)1 << 31)

typedef enum {
    GMM_OK = 0,
    GMM_ERR_INVALID_ARG = 1,   /* bad size, NULL pointer, label or option  */
    GMM_ERR_NOT_SPD = 2,       /* a covariance has a non-positive pivot    */
    GMM_ERR_NONFINITE = 3,     /* NaN/Inf in the points or in a result     */
    GMM_ERR_OOM = 4,           /* workspace too small / allocation failed  */
    GMM_ERR_DEVICE = 5,        /* a HIP runtime call failed                */
    GMM_ERR_UNSUPPORTED = 6    /* a size above the compiled limits         */
} gmm_status;

/* Second-moment accumulation of the M-step.
 *  SHIFTED:  one pass; the E-step's own offsets d = x - mu_old (exact in
 *            FP32 for points near the component) are accumulated as
 *            sum g, sum g d, sum g d d^T (FP32 products, FP64 sums) and
 *            re-centred on the new mean in FP64.
 *  TWO_PASS: a first pass gives the new mean, a second pass (re-deriving
 *            the same responsibilities) accumulates the scatter about it;
 *            twice the E-step work, no re-centring error.                  */
enum { GMM_MOMENTS_SHIFTED = 0, GMM_MOMENTS_TWO_PASS = 1 };

/* flags */
#define GMM_FLAG_ASYNC 1u          /* do not synchronise; read the status later */
#define GMM_FLAG_DETERMINISTIC 2u  /* bitwise reproducible results: every
                                      reduction here has a fixed order, so
                                      this holds for every call (accepted,
                                      changes nothing)                      */

typedef struct {
    int32_t iters;        /* T >= 0 EM iterations (E-step + M-step each)   */
    double reg_covar;     /* lambda >= 0, added to every covariance diagonal
                             after each M-step                             */
    int32_t moment_mode;  /* GMM_MOMENTS_*                                 */
    uint32_t flags;       /* GMM_FLAG_*                                    */
    double tol;           /* >= 0; 0: exactly T iterations (the paper gives
                             no stopping rule).  > 0 (gmm_fit only): after
                             the M-step of iteration t, once
                             |L(theta_t) - L(theta_t-1)| <= tol N the fit
                             keeps theta_t+1 and skips the iterations left
                             (on the device, no host synchronisation): their
                             loglik entries are NaN, loglik[iters] is
                             L(theta_t+1).  Batched and 4D fits need 0.    */
} gmm_fit_opts;

/* Short text of a status code (static storage). */
const char *gmm_status_string(gmm_status s);

/* Text of the last host-side error detected in this thread (static,
 * thread-local; "" when none). */
const char *gmm_last_error(void);

/* Waits for `stream` and returns the device status word of a workspace
 * used by a previous call (GMM_OK when no device-side error was seen). */
gmm_status gmm_workspace_status(const void *ws, void *stream);

/* ---------------------------------------------------------------- fitting
 * gmm_fit: fixed-iteration EM (Sec. V "Expectation Maximization").
 *  pts          device float32 N x 3.
 *  init_labels  device int32 N with values in [0, K), or NULL.  Non-NULL:
 *               theta_0 is the M-step of the one-hot responsibilities these
 *               labels define (the responsibility matrix a k-means style
 *               initialisation hands to EM, Sec. V fig. "information
 *               flow") and w/mu/cov are outputs only.  NULL: w/mu/cov hold
 *               theta_0 on entry.
 *  w, mu, cov   device float32 K, K x 3, K x 3 x 3; theta_T on return.
 *  loglik       device float64 array of iters + 1 entries, or NULL:
 *               loglik[t] = sum_n ln sum_b pi_b N(x_n | mu_b, Sigma_b) at
 *               theta_t (nats; eq. 2 normaliser summed over the points);
 *               loglik[iters] is evaluated at the returned parameters.
 *  Each iteration: E-step with theta_t (FP32 arithmetic, eq. 1-3), M-step
 *  N_b = sum_n g_nb + 10*DBL_EPSILON, pi_b = N_b / sum_a N_a,
 *  mu_b = sum_n g_nb x_n / N_b,
 *  Sigma_b = sum_n g_nb (x_n - mu_b)(x_n - mu_b)^T / N_b + lambda I
 *  (FP64 sums), then an FP64 Cholesky of each Sigma_b for the next E-step.
 *  Internally the staged copy of the points is put in Morton (Z-curve)
 *  order and the E-step skips every (tile of points, component) pair
 *  whose FP32 weights, by a bound over the tile's bounding sphere, are
 *  exactly zero for all of the tile's points, so the results equal the
 *  dense evaluation up to the order of FP32 additions; the caller's arrays are not reordered, and repeated calls
 *  with the same inputs give bitwise identical results.  GMM_CULL=0 or
 *  GMM_SORT=0 in the environment switch the skipping or the ordering off.
 *  Small fits (K <= 16, N <= 65,536 and at most one 256-point tile per
 *  compute unit, shifted moments) skip the ordering and run all soft
 *  iterations in one launch: one block per tile, a device-wide barrier per
 *  iteration, and every block adds all partial rows in the same order and
 *  makes the same FP64 M-step, so the results are again bitwise
 *  reproducible (they differ from the launch-per-pass form in the order of
 *  additions only; GMM_SMALL=0 selects that form).  The barrier waits are
 *  bounded: a block that waits too long gives up, every block exits and
 *  the call returns GMM_ERR_DEVICE.
 *  Synchronises `stream` once at the end unless GMM_FLAG_ASYNC is set.
 *  Errors: INVALID_ARG (sizes, NULL pointers, options), UNSUPPORTED
 *  (K > GMM_MAX_K), OOM (workspace), then device-side NOT_SPD / NONFINITE /
 *  INVALID_ARG (label out of range), DEVICE (a one-launch fit's barrier
 *  gave up, e.g. when other work kept its blocks from being resident). */
size_t gmm_fit_workspace_size(int64_t n, int32_t k, const gmm_fit_opts *opts);

gmm_status gmm_fit(const float *pts, int64_t n, int32_t k,
                   const int32_t *init_labels, float *w, float *mu, float *cov,
                   double *loglik, const gmm_fit_opts *opts, void *ws,
                   size_t ws_bytes, void *stream);

/* ------------------------------------------------ allocation-free fitting
 * gmm_fit_noalloc: gmm_fit for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results and errors as gmm_fit with ws = NULL, except:
 *  - no workspace argument: the workspace lives in one static device array
 *    of GMM_FIT_NOALLOC_MAX_BYTES per GPU, part of the library's code object
 *    (held by every GPU the library runs on until the process ends).  A fit
 *    whose gmm_fit_workspace_size() exceeds it returns GMM_ERR_UNSUPPORTED
 *    before anything is enqueued.
 *  - nothing is allocated: no hipMalloc / hipMallocAsync / hipFree, no
 *    graph capture, no autotuning, no profiling events; the kernels are
 *    launched directly on `stream`, and every value a fit needs zeroed is
 *    cleared by its own kernels at the start of the call.
 *  - always synchronises `stream` once at the end (GMM_FLAG_ASYNC is
 *    GMM_ERR_INVALID_ARG): the status word lives in the shared array, so
 *    the call cannot be recorded into a stream capture.
 *  - every call on one GPU shares that GPU's array: calls that overlap on
 *    one GPU (other host threads, other streams) race and give undefined
 *    results; serialise them. */
#define GMM_FIT_NOALLOC_MAX_BYTES ((size_t)64 << 20)

gmm_status gmm_fit_noalloc(const float *pts, int64_t n, int32_t k,
                           const int32_t *init_labels, float *w, float *mu,
                           float *cov, double *loglik, const gmm_fit_opts *opts,
                           void *stream);

/* --------------------------------------------------------- log-likelihood
 * gmm_loglik: L = sum_n ln sum_b pi_b N(y_n | mu_b, Sigma_b) with
 * y_n = R(omega) x_n + t (eq. 2-3 applied to the transformed cloud).
 *  pose6    device float32 (omega_x, omega_y, omega_z, t_x, t_y, t_z) with
 *           R = exp([omega]_x) (axis-angle), or NULL for the identity.
 *  w        used as given (no renormalisation); must be > 0.
 *  out_L    device float64 scalar.
 *  out_lse  device float32 N (per-point ln sum_b pi_b N(y_n|.)), or NULL.
 *  Does not synchronise.  Errors: host-side as gmm_fit; device-side
 *  NOT_SPD / NONFINITE via gmm_workspace_status(). */
size_t gmm_loglik_workspace_size(int64_t n, int32_t k);

gmm_status gmm_loglik(const float *pts, int64_t n, const float *pose6,
                      int32_t k, const float *w, const float *mu,
                      const float *cov, double *out_L, float *out_lse,
                      void *ws, size_t ws_bytes, void *stream);

/* gmm_loglik_backward: gradient of grad_L * L (the inputs as gmm_loglik).
 *  One pass over the points re-forms the responsibilities (the per-point
 *  normaliser comes with them, so no forward state is needed).
 *  grad_L   device float64 scalar (the upstream gradient), or NULL for 1.
 *  Outputs (device float32, any may be NULL):
 *   g_pose6  6: (dL/domega, dL/dt), omega through the SO(3) left Jacobian;
 *   g_pts    N x 3: dL/dx_n = R^T g_n, g_n = -sum_b gamma_nb Sigma_b^-1 d_nb;
 *   g_w      K: N_b / pi_b (weights treated as free parameters);
 *   g_mu     K x 3: Sigma_b^-1 sum_n gamma_nb d_nb;
 *   g_cov    K x 3 x 3: 1/2 Sigma_b^-1 (sum_n gamma_nb d d^T) Sigma_b^-1
 *            - 1/2 N_b Sigma_b^-1 (the symmetric gradient);
 *  with d_nb = y_n - mu_b and N_b = sum_n gamma_nb.  A component whose
 *  covariance is not SPD sets NOT_SPD in the status word and gets NaN in its
 *  g_w / g_mu / g_cov entries.  Does not synchronise; device-side errors via
 *  gmm_workspace_status(). */
size_t gmm_loglik_backward_workspace_size(int64_t n, int32_t k);

gmm_status gmm_loglik_backward(const float *pts, int64_t n, const float *pose6,
                               int32_t k, const float *w, const float *mu,
                               const float *cov, const double *grad_L,
                               float *g_pose6, float *g_pts, float *g_w,
                               float *g_mu, float *g_cov, void *ws,
                               size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ batching
 * gmm_fit_batched: B independent fits (same options) in one submission.
 *  pts          device float32, the frames' points concatenated (sum N_f x 3).
 *  pt_off       HOST int64 B + 1: frame f owns points [pt_off[f], pt_off[f+1]),
 *               pt_off[0] = 0.
 *  k_off        HOST int32 B + 1: frame f owns components [k_off[f], k_off[f+1]),
 *               k_off[0] = 0; 1 <= K_f <= min(N_f, 512).
 *  init_labels  device int32, concatenated per-frame labels in [0, K_f), or
 *               NULL (then w/mu/cov hold every frame's theta_0).
 *  w, mu, cov   device float32 sum K_f, x 3, x 3 x 3 (concatenated).
 *  loglik       device float64 B x (iters + 1) (row f = frame f), or NULL.
 * Every frame follows gmm_fit exactly (same E-step, M-step and per-frame
 * reductions); a pass over all frames is one tile launch per M-phase class
 * (cost-balanced per-block segments of the frames' tiles), then one
 * reduction and one update launch, with the whole loop captured in a
 * hipGraph.  Launch shape of the soft passes: dense tiles of 64 points with
 * 512 or 1024 threads per block ("bb512", "bb1024"), or culled tiles
 * of 128 points in each frame's Morton order, skipping (tile, component)
 * pairs whose FP32 weights are exactly zero as gmm_fit does ("bc512p8s32",
 * "bc512p8s64", "bc512p16s64").  Default "bb512"; GMM_BATCH_SHAPE=<name>
 * forces one; with autotuning on (gmm_set_autotune), the first call for a
 * new (device, B, K_max, floor(log2 sum N_f K_f)) runs up to 4 EM
 * iterations, times one soft pass of every shape on its own data at that
 * point, keeps the fastest and restarts the fit with it (per process, and in
 * GMM_AUTOTUNE_CACHE as "batch B K_max bucket name" lines).
 * Synchronises once (twice with the plan upload) unless GMM_FLAG_ASYNC.
 * Errors: as gmm_fit, per frame. */
size_t gmm_fit_batched_workspace_size(int32_t B, const int64_t *pt_off,
                                      const int32_t *k_off,
                                      const gmm_fit_opts *opts);

gmm_status gmm_fit_batched(int32_t B, const float *pts, const int64_t *pt_off,
                           const int32_t *k_off, const int32_t *init_labels,
                           float *w, float *mu, float *cov, double *loglik,
                           const gmm_fit_opts *opts, void *ws, size_t ws_bytes,
                           void *stream);

/* The soft-pass shape a gmm_fit_batched call with these frames would use
 * now (static string; "" when autotuning is on and the batch is not tuned
 * yet, or on bad arguments). */
const char *gmm_fit_batched_config(int32_t B, const int64_t *pt_off, const int32_t *k_off);

/* ------------------------------------------------------------ k-means++
 * Seeding of a fit: the paper starts EM from a randomised k-means step
 * (Sec. V); this is k-means++ D^2 seeding (Arthur & Vassilvitskii, 2007),
 * one trial per centre, with hard nearest-centre labels and no Lloyd
 * iterations.  The K random draws are the caller's: u[j] in [0, 1).
 *   centre 0 = floor(u[0] n) (at most n - 1);
 *   centre j = the first point whose running sum of D2 exceeds u[j] W,
 *     D2_i = squared distance from x_i to the nearest earlier centre and
 *     W = sum_i D2_i, so point i is drawn with probability D2_i / W; when
 *     W = 0 (every point on a centre) centre j repeats centre j - 1;
 *   labels[i] = the nearest centre, the lowest j on ties.
 * Distances are ((dx^2 + dy^2) + dz^2) in double, each operation rounded
 * on its own.  The running sums have a fixed order - sequential within
 * chunks of 256 points, chunk totals sequential in runs of 16 from offsets
 * formed by a fixed block scan, inside the chosen chunk a fixed block scan
 * from its running sum; the pick is the first positive entry above u_j W
 * (else the last positive entry) - so the centres are reproducible; where
 * u_j W lies within rounding of a running sum another correct order may
 * pick a neighbouring point.
 *
 * pts: device, n x 3 float32.  u: device, k doubles.  centres: device, k
 * int64 indices into pts (output).  labels: device, n int32 in [0, k)
 * (output; NULL skips the labels).  1 <= k <= min(n, GMM_MAX_K).
 * Synchronises with `stream` once at the end.  Errors: INVALID_ARG (sizes,
 * NULL pointers, a draw outside [0, 1)), NONFINITE (a non-finite point),
 * OOM / DEVICE as for the other entry points; the outputs are unspecified
 * after an error. */
size_t gmm_kmeanspp_workspace_size(int64_t n, int32_t k);
gmm_status gmm_kmeanspp(const float *pts, int64_t n, int32_t k, const double *u,
                        int64_t *centres, int32_t *labels, void *ws, size_t ws_bytes,
                        void *stream);

/* ------------------------------------------- 4D model: position + intensity
 * The paper's model (Sec. IV "GIRA Reconstruction"; Sec. V tensor shapes:
 * weights (1, K, 1), means (1, K, 4), covariances (1, K, 4, 4)) is a
 * mixture over 4D points (x, y, z, intensity); its size is
 * 4 K (1 + 4 + 10) bytes in float32.
 *
 * gmm4_fit: fixed-iteration EM of the 4D mixture, exactly as gmm_fit with
 * D = 4 (eq. 1-3 with D ln 2pi / 2 = 2 ln 2pi; M-step N_b = sum g + 10
 * DBL_EPSILON, pi_b = N_b / sum N, mu_b = sum g x / N_b, Sigma_b = sum g
 * (x - mu)(x - mu)^T / N_b + lambda I; FP32 E-step, FP64 sums, FP64 4 x 4
 * Cholesky).  The soft passes take the points in Morton order of their
 * xyz part (a copy in the workspace) and skip the (64-point tile,
 * component) pairs whose FP32 weight is zero for the whole tile, bounded by
 * the xyz marginal of the component; the result is the dense evaluation's
 * up to the order of floating-point additions.  GMM_CULL4=0 evaluates every
 * pair in the caller's order; the workspace size depends on that setting.
 *  pts          device float32 N x 4 (x, y, z, intensity), 16-byte aligned.
 *  init_labels  device int32 N in [0, K), or NULL (then w/mu/cov hold
 *               theta_0 on entry, weights used as given).
 *  w, mu, cov   device float32 K, K x 4, K x 4 x 4 (lower triangle read,
 *               symmetric written); theta_T on return.
 *  loglik       device float64 iters + 1 entries, or NULL (as gmm_fit).
 *  1 <= K <= 512, K <= N.  Synchronises once unless GMM_FLAG_ASYNC (then
 *  the status word is at the start of ws: gmm_workspace_status).
 *  Errors: as gmm_fit; points not 16-byte aligned are INVALID_ARG. */
size_t gmm4_fit_workspace_size(int64_t n, int32_t k, const gmm_fit_opts *opts);
gmm_status gmm4_fit(const float *pts, int64_t n, int32_t k, const int32_t *init_labels,
                    float *w, float *mu, float *cov, double *loglik,
                    const gmm_fit_opts *opts, void *ws, size_t ws_bytes, void *stream);

/* gmm4_color_conditional: expected intensity and its variance at known 3D
 * locations (the paper's color_conditional).  Under the 4D mixture the
 * intensity given x is a mixture of 1D Gaussians: weights beta_b(x)
 * proportional to pi_b N(x | mu_b^x, Sigma_b^xx) (3D marginals), means
 * m_b(x) = mu_b^i + Sigma_b^ix (Sigma_b^xx)^-1 (x - mu_b^x), variances
 * v_b = Sigma_b^ii - Sigma_b^ix (Sigma_b^xx)^-1 Sigma_b^xi; expected[i] =
 * sum_b beta_b m_b and variance[i] = sum_b beta_b (v_b + m_b^2) - E^2.
 *  locs      device float32 M x 3;  expected, variance: device float32 M.
 *  w, mu, cov  the 4D mixture as gmm4_fit returns it (w > 0).
 *  FP32 per (location, component) terms, FP64 sums; FP64 Cholesky per
 *  component.  Does not synchronise; device-side NOT_SPD / NONFINITE /
 *  INVALID_ARG (w <= 0) via gmm_workspace_status(ws).  1 <= K <= 512. */
size_t gmm4_color_conditional_workspace_size(int32_t k);
gmm_status gmm4_color_conditional(const float *locs, int64_t m, int32_t k, const float *w,
                                  const float *mu, const float *cov, float *expected,
                                  float *variance, void *ws, size_t ws_bytes, void *stream);

/* gmm4_joint_dist_sample: M samples of the 4D mixture (the paper's
 * joint_dist_sample) from caller-given draws: sample s takes the first
 * component whose running sum of the weights (component order, FP64)
 * exceeds u[s] W, W the total (the last component with w > 0 when rounding
 * leaves none), and is mu_b + L_b z[s] with Sigma_b = L_b L_b^T (FP64
 * Cholesky, FP64 arithmetic, rounded to float32).
 *  u     device float64 M in [0, 1);  z: device float32 M x 4 standard
 *        normals;  out: device float32 M x 4;  comp: device int32 M (the
 *        chosen components) or NULL.
 *  w >= 0 with a positive total.  Does not synchronise; device-side errors
 *  (a draw outside [0, 1), w < 0, a covariance not SPD) via
 *  gmm_workspace_status(ws).  1 <= K <= GMM_MAX_K. */
size_t gmm4_joint_dist_sample_workspace_size(int32_t k);
gmm_status gmm4_joint_dist_sample(int32_t k, const float *w, const float *mu, const float *cov,
                                  int64_t m, const double *u, const float *z, float *out,
                                  int32_t *comp, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ autotuning
 * With autotuning on (gmm_set_autotune(1), or GMM_AUTOTUNE=1 in the
 * environment), the first gmm_fit for a new (device arch, K, N bucket =
 * floor(log2 N)) times every tile shape the library can run on one E+M pass
 * of the caller's own data (the parameters are not changed by it), keeps
 * the fastest for this process and, when GMM_AUTOTUNE_CACHE names a file,
 * appends "arch K bucket shape" lines to it and reads it back next time.
 * GMM_TILE_SHAPE=<name> in the environment forces one shape when it can
 * run the given K.  gmm_tile_config returns the shape a call with (n, k)
 * would use now (static string, "" on bad sizes). */
gmm_status gmm_set_autotune(int on);
const char *gmm_tile_config(int64_t n, int32_t k);

/* ---------------------------------------------------- component count
 * gmm_meanshift: the number of mixture components K for a bandwidth h, by
 * mean shift with a flat kernel over binned seeds (the paper, Sec. V
 * "Gaussian Blurring Mean Shift", and its information-flow figure, where the
 * bandwidth and the point cloud give K before k-means seeding and EM):
 *   seeds   the centres b h of the occupied bins b = rint(x / h) (FP64
 *           division, round half to even), in lexicographic order of b;
 *   shift   a seed moves to the mean of the points within distance h
 *           (squared distance ((d0^2 + d1^2) + d2^2) (+ d3^2) <= h^2, every
 *           FP64 operation rounded on its own) until the move is at most
 *           1e-3 h or its iteration count has reached max_iter; its weight
 *           is the size of the last neighbourhood (0 when the first one is
 *           empty: the seed is dropped);
 *   merge   in the order (weight descending, coordinates descending, seed
 *           ascending) a mode still kept removes every later mode within
 *           h; K is the number kept.
 *  pts          device float32 n x d: d = 3 (x, y, z) or d = 4 (x, y, z,
 *               intensity).  Every bin index |rint(x / h)| must be at most
 *               2^20 - 2 (d = 3) or 2^15 - 2 (d = 4), else INVALID_ARG.
 *  bandwidth    h, finite and > 0.   max_iter >= 0 (a seed takes at most
 *               max_iter + 1 means).
 *  modes        device float64 max_modes x d: the kept modes, in seed order;
 *  weights      device int64 max_modes, or NULL: their weights.  More than
 *               max_modes kept is INVALID_ARG, with info->n_modes set
 *               (max_modes = n always suffices).
 *  seed_modes   device float64 n x d; seed_weights, seed_iters, seed_status:
 *               device int32 n.  Each NULL, or filled for the
 *               info->n_seeds seeds: mode, weight, iteration count, and
 *               1 kept / 2 removed by the merge / 3 dropped.
 *  info         host: seeds, K, merge rounds, largest iteration count.
 *  Synchronises: the merge checks its progress on the host every 16 rounds
 *  and the call returns K.  n = 0 gives K = 0.  FP64 sums in a fixed order
 *  (one wave per seed, or four when there are at most 16,384 seeds; the
 *  order depends only on the cells of a neighbourhood): modes, weights and
 *  K are bitwise reproducible; the number of merge rounds may differ
 *  between calls (a round can see decisions made earlier in the same
 *  round).  Errors: INVALID_ARG (d, n, h, max_iter, NULL
 *  pointers, bin range), NONFINITE (a NaN or Inf coordinate), OOM, DEVICE. */
typedef struct {
    int64_t n_seeds;    /* occupied bins */
    int32_t n_modes;    /* K */
    int32_t rounds;     /* merge rounds until every mode was decided (may vary) */
    int32_t max_iters;  /* the largest iteration count of a seed */
} gmm_meanshift_info;
size_t gmm_meanshift_workspace_size(int64_t n, int32_t d);
gmm_status gmm_meanshift(const float *pts, int64_t n, int32_t d, double bandwidth,
                         int32_t max_iter, double *modes, int64_t *weights, int64_t max_modes,
                         double *seed_modes, int32_t *seed_weights, int32_t *seed_iters,
                         int32_t *seed_status, gmm_meanshift_info *info, void *ws,
                         size_t ws_bytes, void *stream);

/* --------------------------------------- registration of two mixtures
 * Distribution-to-distribution (D2D) registration of a source mixture
 * (pi_i, mu_i, Sigma_i), i < M, to a target mixture (tau_j, nu_j,
 * Lambda_j), j < N: the paper's GIRA Registration (Sec. IV) with its
 * anisotropic, isoplanar and isoplanar-then-anisotropic variants, whose
 * formulas the paper leaves to its citation.  The objective is
 *   f(T) = ln sum_ij pi_i tau_j N(R mu_i + t; nu_j, R Sigma_i R^T + Lambda_j),
 * the log of the integral of the product of the transformed source density
 * and the target density; isoplanar replaces every covariance by
 * I - (1 - 1e-3) v v^T, v the eigenvector of its smallest eigenvalue.
 * All arithmetic is FP64 (inputs are float32 mixtures as the fits return
 * them); sums are in a fixed order (bitwise reproducible).
 *  w, mu, cov / tw, tmu, tcov  device float32 M, M x 3, M x 3 x 3 (lower
 *              triangle read) and N, N x 3, N x 3 x 3; weights > 0.
 *  1 <= M, N <= 65535.  Neither call synchronises: device-side errors (a
 *  weight <= 0: INVALID_ARG; S_ij not positive definite: NOT_SPD; a
 *  non-finite value: NONFINITE) are read with gmm_workspace_status(ws). */
#define GMM_D2D_ANISOTROPIC 0
#define GMM_D2D_ISOPLANAR 1
size_t gmm_d2d_workspace_size(int32_t m, int32_t n);
/* gmm_d2d_objective: f and its gradient at one pose.
 *  pose6     device float64 6: (omega, t), R = exp([omega]_x) (Rodrigues).
 *  variant   GMM_D2D_ANISOTROPIC or GMM_D2D_ISOPLANAR.
 *  out       device float64 7: f, df/domega (3), df/dt (3); df/domega =
 *            J_l(omega)^T df/ddelta for a left perturbation exp([delta]_x) R. */
gmm_status gmm_d2d_objective(const double *pose6, int32_t m, const float *w, const float *mu,
                             const float *cov, int32_t n, const float *tw, const float *tmu,
                             const float *tcov, int32_t variant, double *out, void *ws,
                             size_t ws_bytes, void *stream);
/* gmm_d2d_register: iters_iso isoplanar iterations, then iters_aniso
 * anisotropic ones (either may be 0: the pure variants), from T0.  An
 * iteration: H = sum_ij gamma_ij J^T S_ij^-1 J (gamma_ij the pair's share of
 * the sum at T, J = [-[R mu_i]_x, I], S_ij at T), x = H^-1 grad f (FP64
 * Cholesky; grad in (delta, t)), then the first of R' = exp([s x_w]_x) R,
 * t' = t + s x_t, s = 1, 1/2, ..., 2^-7, with f(T') > f(T).  A stage ends
 * early when H is not positive definite, max |x| < 1e-8 or no trial
 * increases f.
 *  T0, T_out   device float64 4 x 4 row-major transforms (T_out = [R t; 0 1]).
 *  history     device float64 iters_iso + iters_aniso + 2, or NULL: f at the
 *              start of each stage and after every accepted iteration, in
 *              order, NaN after the last.
 *  counts      device int32 2, or NULL: accepted iterations per stage. */
gmm_status gmm_d2d_register(const double *T0, int32_t m, const float *w, const float *mu,
                            const float *cov, int32_t n, const float *tw, const float *tmu,
                            const float *tcov, int32_t iters_iso, int32_t iters_aniso,
                            double *T_out, double *history, int32_t *counts, void *ws,
                            size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ profiling
 * Kernel timing for benchmarks.  While enabled (reps >= 1, per calling host
 * thread), every E+M statistics pass of the tile kernel made by gmm_fit, the
 * tile pass of gmm_loglik and the backward tile kernel of
 * gmm_loglik_backward are launched reps times back to back between two HIP
 * events recorded on the caller's stream (such calls launch their kernels
 * directly instead of replaying a captured graph).  These kernels only read
 * the points and parameters and overwrite their own outputs and partial
 * sums, so the repeats change no result; they spread the event pair's
 * dispatch latency (a few microseconds) over reps launches.  reps = 0 disables; reps > 64 is
 * INVALID_ARG.  gmm_profile_read waits for the recorded events, returns the
 * summed elapsed time (ms) and the number of tile launches it covers since
 * the last read, and resets both.  Errors: DEVICE when an event call fails. */
gmm_status gmm_profile_enable(int reps);
gmm_status gmm_profile_read(double *tile_ms_total, int64_t *tile_launches);
/* The (tile, component) pairs of the timed E+M launches since the last
 * call: `all` = launches x tiles x K, `evaluated` = the pairs the kernels
 * computed (all of them for a dense tile kernel; for the culled kernel,
 * those its bound could not show to be exactly zero).  Waits for the
 * device; resets both.  Errors: DEVICE. */
gmm_status gmm_profile_pairs(int64_t *evaluated, int64_t *all);

#ifdef __cplusplus
}
#endif

#endif /* GMM_MI355X_H */
