/* Drives every entry point of the C oracle on a small synthetic cloud, for
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitize.py): any out-of-bounds access, leak or undefined
 * operation aborts the program.  Returns 0 when every call succeeds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_component_terms(int K, const double *w, const double *cov, double *P, double *c);
int oracle_estep(int64_t N, const double *X, int K, const double *w, const double *mu,
                 const double *cov, double *lse_out, double *logresp_out, double *L_out);
int oracle_mstep_labels(int64_t N, const double *X, const int32_t *labels, int K, double reg,
                        double *w, double *mu, double *cov);
int oracle_em_step(int64_t N, const double *X, int K, const double *w_in, const double *mu_in,
                   const double *cov_in, double reg, double *w_out, double *mu_out,
                   double *cov_out, double *L_in);
int oracle_fit(int64_t N, const double *X, int K, const int32_t *labels, double *w, double *mu,
               double *cov, double reg, int T, double *Lhist);
int oracle_loglik_pose(int64_t N, const double *X, const double *pose6, int K, const double *w,
                       const double *mu, const double *cov, double *L_out, double *lse_out);
int oracle_loglik_grad(int64_t N, const double *X, const double *pose6, int K, const double *w,
                       const double *mu, const double *cov, double grad_L, double *g_pose6,
                       double *g_pts, double *g_w, double *g_mu, double *g_cov);
int oracle_nearest(int64_t N, const double *X, int K, const int64_t *centres, int32_t *labels);
int oracle_kmeanspp(int64_t N, const double *X, int K, const double *u, int64_t *centres,
                    int32_t *labels);
int oracle_kmeanspp_replay(int64_t N, const double *X, int K, const double *u,
                           const int64_t *centres, int64_t *flat_pick, double *W2,
                           double *before2, double *at2);

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double urand(void) {  /* xorshift64*, [0, 1) */
  g_state ^= g_state >> 12;
  g_state ^= g_state << 25;
  g_state ^= g_state >> 27;
  return (double)((g_state * 2685821657736338717ull) >> 11) * 0x1p-53;
}

#define CHECK(call)                                                 \
  do {                                                              \
    int st_ = (call);                                               \
    if (st_ != 0) {                                                 \
      fprintf(stderr, "%s failed with %d\n", #call, st_);           \
      return 1;                                                     \
    }                                                               \
  } while (0)

int main(void) {
  const int64_t N = 3001;
  const int K = 7, T = 4;
  double *X = malloc(sizeof(double) * 3 * N);
  int32_t *lab = malloc(sizeof(int32_t) * N);
  for (int64_t i = 0; i < N; ++i) {
    const int c = (int)(i % K);
    for (int j = 0; j < 3; ++j) X[3 * i + j] = 2.0 * c + (j == 0 ? 3.0 : 1.0) * (urand() - 0.5);
    lab[i] = c;
  }
  double w[7], mu[21], cov[63], Lh[T + 1], P[63], c[7], w2[7], mu2[21], cov2[63], L = 0.0;
  double *lse = malloc(sizeof(double) * N), *lr = malloc(sizeof(double) * N * K);
  double *gp = malloc(sizeof(double) * 3 * N);
  CHECK(oracle_mstep_labels(N, X, lab, K, 1e-3, w, mu, cov));
  CHECK(oracle_component_terms(K, w, cov, P, c));
  CHECK(oracle_estep(N, X, K, w, mu, cov, lse, lr, &L));
  CHECK(oracle_em_step(N, X, K, w, mu, cov, 1e-3, w2, mu2, cov2, &L));
  CHECK(oracle_fit(N, X, K, lab, w, mu, cov, 1e-3, T, Lh));
  const double pose[6] = {0.1, -0.2, 0.05, 0.3, 0.0, -0.1};
  double gpose[6], gw[7], gmu[21], gcov[63];
  CHECK(oracle_loglik_pose(N, X, pose, K, w, mu, cov, &L, lse));
  CHECK(oracle_loglik_grad(N, X, pose, K, w, mu, cov, 1.5, gpose, gp, gw, gmu, gcov));
  CHECK(oracle_loglik_grad(N, X, NULL, K, w, mu, cov, 1.0, NULL, NULL, gw, NULL, NULL));
  double u[7];
  for (int j = 0; j < K; ++j) u[j] = urand();
  int64_t cen[7], flat[7];
  double W2[14], b2[14], a2[14];
  CHECK(oracle_kmeanspp(N, X, K, u, cen, lab));
  CHECK(oracle_nearest(N, X, K, cen, lab));
  CHECK(oracle_kmeanspp_replay(N, X, K, u, cen, flat, W2, b2, a2));
  int bad = 0;
  for (int j = 0; j < K; ++j) bad |= flat[j] != cen[j];
  for (int t = 0; t <= T; ++t) bad |= !isfinite(Lh[t]);
  /* an argument error is reported, not acted on */
  bad |= oracle_fit(0, X, K, lab, w, mu, cov, 1e-3, T, Lh) == 0;
  free(X); free(lab); free(lse); free(lr); free(gp);
  if (bad) {
    fprintf(stderr, "unexpected results\n");
    return 1;
  }
  printf("oracle driver ok\n");
  return 0;
}
