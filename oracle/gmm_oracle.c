/*
 * FP64 CPU oracle for 3D Gaussian-mixture EM and the point-cloud GMM
 * log-likelihood.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke
 * check and the benchmark's CPU-baseline leg are its only users.  It shares
 * no code, header, constant or helper with the HIP library; nothing in the
 * product path may load it.
 *
 * Everything is written as the plain definition, in double precision,
 * one point and one component at a time:
 *
 *   E-step  (paper Sec. V "Expectation Maximization", eq. 1-3)
 *     Sigma_b = L_b L_b^T (Cholesky), P_b = L_b^{-1}
 *     ln N(x | mu_b, Sigma_b) = -1/2 (D ln 2pi + |P_b (x - mu_b)|^2)
 *                               + sum_j ln (P_b)_jj                   (eq. 3)
 *     l_nb   = ln pi_b + ln N(x_n | mu_b, Sigma_b)
 *     lse_n  = ln sum_a exp(l_na)          (max-shifted)             (eq. 2)
 *     gamma_nb = exp(l_nb - lse_n)                                   (eq. 1)
 *     L      = sum_n lse_n      (log-likelihood, nats)
 *
 *   M-step  (the paper names it but prints no formulas; this is the
 *   standard maximum-likelihood update for full covariances, with the
 *   conventions listed in the design notes):
 *     N_b     = sum_n gamma_nb + eps_N,            eps_N = 10 * DBL_EPSILON
 *     pi_b    = N_b / sum_a N_a
 *     mu_b    = sum_n gamma_nb x_n / N_b
 *     Sigma_b = sum_n gamma_nb (x_n - mu_b)(x_n - mu_b)^T / N_b + lambda I
 *   computed with an exact two-pass centring (pass 1: N_b, mu_b; pass 2:
 *   the centred second moment, re-deriving gamma from the same theta).
 *
 *   Registration log-likelihood: y_n = R(omega) x_n + t (Rodrigues'
 *   formula for R), L = sum_n lse_n(y_n), and its analytic gradient with
 *   respect to pose, points, weights, means and covariances.
 *
 * Reductions over points use OpenMP with per-thread partial sums merged in
 * thread order (a static schedule), so a run is reproducible for a given
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_NOT_SPD 2
#define OR_ERR_NONFINITE 3
#define OR_ERR_OOM 4

static const double OR_LN_2PI = 1.8378770664093454835606594728112;
static const double OR_EPS_N = 10.0 * 2.220446049250313080847263336181640625e-16;

/* ---- thread control ---------------------------------------------------- */

void oracle_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}

int oracle_get_threads(void) { return omp_get_max_threads(); }

/* ---- 3x3 helpers (row-major, lower triangle used) ----------------------- */

/* Cholesky factor L (lower, row-major 3x3) of the symmetric matrix whose
 * lower triangle is A.  Returns 0 on success, -1 when a pivot is not
 * strictly positive or not finite. */
static int chol3(const double *A, double *L) {
    memset(L, 0, 9 * sizeof(double));
    for (int j = 0; j < 3; ++j) {
        double s = A[j * 3 + j];
        for (int k = 0; k < j; ++k) s -= L[j * 3 + k] * L[j * 3 + k];
        if (!(s > 0.0) || !isfinite(s)) return -1;
        double d = sqrt(s);
        L[j * 3 + j] = d;
        for (int i = j + 1; i < 3; ++i) {
            double t = A[i * 3 + j];
            for (int k = 0; k < j; ++k) t -= L[i * 3 + k] * L[j * 3 + k];
            L[i * 3 + j] = t / d;
        }
    }
    return 0;
}

/* Inverse of a lower-triangular 3x3 matrix by forward substitution on the
 * identity: column c of P solves L p = e_c. */
static void tri_inv3(const double *L, double *P) {
    memset(P, 0, 9 * sizeof(double));
    for (int c = 0; c < 3; ++c) {
        for (int i = c; i < 3; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= L[i * 3 + k] * P[k * 3 + c];
            P[i * 3 + c] = s / L[i * 3 + i];
        }
    }
}

/* Per-component terms of eq. 3: precision Cholesky P_b = L_b^{-1} and the
 * constant c_b = ln pi_b - (D/2) ln 2pi + sum_j ln (P_b)_jj. */
int oracle_component_terms(int K, const double *w, const double *cov,
                           double *P, double *c) {
    if (K <= 0 || !w || !cov || !P || !c) return OR_ERR_ARG;
    for (int b = 0; b < K; ++b) {
        double L[9];
        if (!(w[b] > 0.0) || !isfinite(w[b])) return OR_ERR_ARG;
        if (chol3(cov + 9 * b, L) != 0) return OR_ERR_NOT_SPD;
        tri_inv3(L, P + 9 * b);
        double logdiag = 0.0;
        for (int j = 0; j < 3; ++j) logdiag += log(P[9 * b + j * 3 + j]);
        c[b] = log(w[b]) - 0.5 * 3.0 * OR_LN_2PI + logdiag;
    }
    return OR_OK;
}

/* l_nb for one point and all components (eq. 2-3). */
static void point_logterms(const double *x, int K, const double *mu,
                           const double *P, const double *c, double *l) {
    for (int b = 0; b < K; ++b) {
        const double *m = mu + 3 * b;
        const double *p = P + 9 * b;
        double d0 = x[0] - m[0], d1 = x[1] - m[1], d2 = x[2] - m[2];
        double z0 = p[0] * d0;
        double z1 = p[3] * d0 + p[4] * d1;
        double z2 = p[6] * d0 + p[7] * d1 + p[8] * d2;
        l[b] = c[b] - 0.5 * (z0 * z0 + z1 * z1 + z2 * z2);
    }
}

/* Max-shifted log-sum-exp over the K terms, and the responsibilities
 * gamma_b = exp(l_b - lse) when g is non-NULL (eq. 1-2). */
static double point_lse(int K, const double *l, double *g) {
    double m = l[0];
    for (int b = 1; b < K; ++b)
        if (l[b] > m) m = l[b];
    double s = 0.0;
    for (int b = 0; b < K; ++b) s += exp(l[b] - m);
    double lse = m + log(s);
    if (g)
        for (int b = 0; b < K; ++b) g[b] = exp(l[b] - lse);
    return lse;
}

/* ---- E-step -------------------------------------------------------------- */

/* lse_n (may be NULL), the full log-responsibility matrix ln gamma (N x K,
 * may be NULL; intended for small inputs) and L = sum_n lse_n. */
int oracle_estep(int64_t N, const double *X, int K, const double *w,
                 const double *mu, const double *cov, double *lse_out,
                 double *logresp_out, double *L_out) {
    if (N < 0 || K <= 0 || (N > 0 && !X) || !L_out) return OR_ERR_ARG;
    double *P = malloc(sizeof(double) * 9 * K);
    double *c = malloc(sizeof(double) * K);
    if (!P || !c) { free(P); free(c); return OR_ERR_OOM; }
    int st = oracle_component_terms(K, w, cov, P, c);
    if (st != OR_OK) { free(P); free(c); return st; }
    int nt = omp_get_max_threads();
    double *Lpart = calloc(nt, sizeof(double));
    int bad = 0;
#pragma omp parallel
    {
        int tid = omp_get_thread_num();
        double *l = malloc(sizeof(double) * K);
        double acc = 0.0;
#pragma omp for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            point_logterms(X + 3 * n, K, mu, P, c, l);
            double v = point_lse(K, l, NULL);
            if (lse_out) lse_out[n] = v;
            if (logresp_out)
                for (int b = 0; b < K; ++b) logresp_out[n * K + b] = l[b] - v;
            acc += v;
        }
        Lpart[tid] = acc;
        free(l);
    }
    double L = 0.0;
    for (int t = 0; t < nt; ++t) L += Lpart[t];
    if (!isfinite(L)) bad = 1;
    *L_out = L;
    free(Lpart); free(P); free(c);
    return bad ? OR_ERR_NONFINITE : OR_OK;
}

/* ---- M-step ---------------------------------------------------------------
 * Responsibilities come either from theta (soft, eq. 1) or from hard labels
 * (one-hot, the responsibility matrix of a k-means initialisation).  The
 * update is the same in both cases. */

typedef struct {
    int K;
    const double *mu, *P, *c;   /* soft mode */
    const int32_t *labels;      /* hard mode */
} resp_src;

/* Responsibilities of point n; returns lse_n (0 in hard mode). */
static double point_resp(const resp_src *src, int64_t n, const double *x,
                         double *l, double *g) {
    if (src->labels) {
        for (int b = 0; b < src->K; ++b) g[b] = 0.0;
        g[src->labels[n]] = 1.0;
        return 0.0;
    }
    point_logterms(x, src->K, src->mu, src->P, src->c, l);
    return point_lse(src->K, l, g);
}

static int mstep_two_pass(int64_t N, const double *X, const resp_src *src,
                          double reg, double *w_out, double *mu_out,
                          double *cov_out, double *L_out) {
    const int K = src->K;
    int nt = omp_get_max_threads();
    /* per-thread partials: [N0, sx0, sx1, sx2] per component, then 6 */
    double *p1 = calloc((size_t)nt * K * 4, sizeof(double));
    double *p2 = calloc((size_t)nt * K * 6, sizeof(double));
    double *Lp = calloc(nt, sizeof(double));
    double *Nb = malloc(sizeof(double) * K);
    double *mu = malloc(sizeof(double) * 3 * K);
    if (!p1 || !p2 || !Lp || !Nb || !mu) {
        free(p1); free(p2); free(Lp); free(Nb); free(mu);
        return OR_ERR_OOM;
    }
    /* pass 1: N_b and sum gamma x */
#pragma omp parallel
    {
        int tid = omp_get_thread_num();
        double *l = malloc(sizeof(double) * K), *g = malloc(sizeof(double) * K);
        double *a = p1 + (size_t)tid * K * 4;
        double acc = 0.0;
#pragma omp for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            const double *x = X + 3 * n;
            acc += point_resp(src, n, x, l, g);
            for (int b = 0; b < K; ++b) {
                a[4 * b + 0] += g[b];
                a[4 * b + 1] += g[b] * x[0];
                a[4 * b + 2] += g[b] * x[1];
                a[4 * b + 3] += g[b] * x[2];
            }
        }
        Lp[tid] = acc;
        free(l); free(g);
    }
    double Ntot = 0.0;
    for (int b = 0; b < K; ++b) {
        double s[4] = {0, 0, 0, 0};
        for (int t = 0; t < nt; ++t)
            for (int j = 0; j < 4; ++j) s[j] += p1[((size_t)t * K + b) * 4 + j];
        Nb[b] = s[0] + OR_EPS_N;
        for (int j = 0; j < 3; ++j) mu[3 * b + j] = s[j + 1] / Nb[b];
        Ntot += Nb[b];
    }
    /* pass 2: centred second moment about the new means */
#pragma omp parallel
    {
        int tid = omp_get_thread_num();
        double *l = malloc(sizeof(double) * K), *g = malloc(sizeof(double) * K);
        double *a = p2 + (size_t)tid * K * 6;
#pragma omp for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            const double *x = X + 3 * n;
            point_resp(src, n, x, l, g);
            for (int b = 0; b < K; ++b) {
                double d0 = x[0] - mu[3 * b], d1 = x[1] - mu[3 * b + 1],
                       d2 = x[2] - mu[3 * b + 2];
                a[6 * b + 0] += g[b] * d0 * d0;
                a[6 * b + 1] += g[b] * d1 * d0;
                a[6 * b + 2] += g[b] * d1 * d1;
                a[6 * b + 3] += g[b] * d2 * d0;
                a[6 * b + 4] += g[b] * d2 * d1;
                a[6 * b + 5] += g[b] * d2 * d2;
            }
        }
        free(l); free(g);
    }
    for (int b = 0; b < K; ++b) {
        double s[6] = {0, 0, 0, 0, 0, 0};
        for (int t = 0; t < nt; ++t)
            for (int j = 0; j < 6; ++j) s[j] += p2[((size_t)t * K + b) * 6 + j];
        double *C = cov_out + 9 * b;
        C[0] = s[0] / Nb[b] + reg;
        C[3] = C[1] = s[1] / Nb[b];
        C[4] = s[2] / Nb[b] + reg;
        C[6] = C[2] = s[3] / Nb[b];
        C[7] = C[5] = s[4] / Nb[b];
        C[8] = s[5] / Nb[b] + reg;
        w_out[b] = Nb[b] / Ntot;
        for (int j = 0; j < 3; ++j) mu_out[3 * b + j] = mu[3 * b + j];
    }
    double L = 0.0;
    for (int t = 0; t < nt; ++t) L += Lp[t];
    if (L_out) *L_out = L;
    free(p1); free(p2); free(Lp); free(Nb); free(mu);
    return OR_OK;
}

/* M-step from hard labels in [0, K) (one-hot responsibilities). */
int oracle_mstep_labels(int64_t N, const double *X, const int32_t *labels,
                        int K, double reg, double *w, double *mu, double *cov) {
    if (N <= 0 || K <= 0 || !X || !labels || !w || !mu || !cov || !(reg >= 0))
        return OR_ERR_ARG;
    for (int64_t n = 0; n < N; ++n)
        if (labels[n] < 0 || labels[n] >= K) return OR_ERR_ARG;
    resp_src src = {K, NULL, NULL, NULL, labels};
    return mstep_two_pass(N, X, &src, reg, w, mu, cov, NULL);
}

/* One EM iteration: E-step with theta_in (its log-likelihood goes to
 * *L_in), then the M-step giving theta_out.  In and out may alias. */
int oracle_em_step(int64_t N, const double *X, int K, const double *w_in,
                   const double *mu_in, const double *cov_in, double reg,
                   double *w_out, double *mu_out, double *cov_out,
                   double *L_in) {
    if (N <= 0 || K <= 0 || !X || !(reg >= 0)) return OR_ERR_ARG;
    double *P = malloc(sizeof(double) * 9 * K);
    double *c = malloc(sizeof(double) * K);
    double *mu = malloc(sizeof(double) * 3 * K);
    if (!P || !c || !mu) { free(P); free(c); free(mu); return OR_ERR_OOM; }
    int st = oracle_component_terms(K, w_in, cov_in, P, c);
    if (st == OR_OK) {
        memcpy(mu, mu_in, sizeof(double) * 3 * K);
        resp_src src = {K, mu, P, c, NULL};
        double L;
        st = mstep_two_pass(N, X, &src, reg, w_out, mu_out, cov_out, &L);
        if (L_in) *L_in = L;
        if (st == OR_OK && !isfinite(L)) st = OR_ERR_NONFINITE;
    }
    free(P); free(c); free(mu);
    return st;
}

/* Fixed-iteration EM fit.  With labels, theta_0 is the M-step of the
 * one-hot responsibilities and (w, mu, cov) are outputs only; without,
 * (w, mu, cov) hold theta_0 on entry.  On exit they hold theta_T, and
 * Lhist[t] = L(theta_t) for t = 0..T (T+1 entries; may be NULL). */
int oracle_fit(int64_t N, const double *X, int K, const int32_t *labels,
               double *w, double *mu, double *cov, double reg, int T,
               double *Lhist) {
    if (N <= 0 || K <= 0 || T < 0 || !X || !w || !mu || !cov) return OR_ERR_ARG;
    int st;
    if (labels) {
        st = oracle_mstep_labels(N, X, labels, K, reg, w, mu, cov);
        if (st != OR_OK) return st;
    }
    for (int t = 0; t < T; ++t) {
        double L;
        st = oracle_em_step(N, X, K, w, mu, cov, reg, w, mu, cov, &L);
        if (Lhist) Lhist[t] = L;
        if (st != OR_OK) return st;
    }
    double L;
    st = oracle_estep(N, X, K, w, mu, cov, NULL, NULL, &L);
    if (Lhist) Lhist[T] = L;
    return st;
}

/* ---- registration log-likelihood -------------------------------------------
 * pose6 = (omega_x, omega_y, omega_z, t_x, t_y, t_z); R = exp([omega]_x). */

static void skew3(const double *v, double *S) {
    S[0] = 0.0;   S[1] = -v[2]; S[2] = v[1];
    S[3] = v[2];  S[4] = 0.0;   S[5] = -v[0];
    S[6] = -v[1]; S[7] = v[0];  S[8] = 0.0;
}

static void matmul3(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
            C[i * 3 + j] = s;
        }
}

/* Rodrigues: R = I + a [w]_x + b [w]_x^2 with a = sin(th)/th and
 * b = (1 - cos th)/th^2; both by their Taylor series when th is tiny. */
static void rodrigues(const double *wv, double *R) {
    double th2 = wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2];
    double th = sqrt(th2), a, b;
    if (th < 1e-4) {
        a = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / th2;
    }
    double S[9], S2[9];
    skew3(wv, S);
    matmul3(S, S, S2);
    for (int i = 0; i < 9; ++i) R[i] = a * S[i] + b * S2[i];
    R[0] += 1.0; R[4] += 1.0; R[8] += 1.0;
}

/* Left Jacobian of SO(3): J = I + b [w]_x + e [w]_x^2 with
 * b = (1 - cos th)/th^2, e = (th - sin th)/th^3. */
static void so3_left_jacobian(const double *wv, double *J) {
    double th2 = wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2];
    double th = sqrt(th2), b, e;
    if (th < 1e-4) {
        b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        e = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        b = (1.0 - cos(th)) / th2;
        e = (th - sin(th)) / (th2 * th);
    }
    double S[9], S2[9];
    skew3(wv, S);
    matmul3(S, S, S2);
    for (int i = 0; i < 9; ++i) J[i] = b * S[i] + e * S2[i];
    J[0] += 1.0; J[4] += 1.0; J[8] += 1.0;
}

static void transform_point(const double *R, const double *t, const double *x,
                            double *y) {
    for (int i = 0; i < 3; ++i)
        y[i] = R[i * 3] * x[0] + R[i * 3 + 1] * x[1] + R[i * 3 + 2] * x[2] + t[i];
}

/* L(pose) = sum_n lse_n(R x_n + t); pose6 NULL means identity. */
int oracle_loglik_pose(int64_t N, const double *X, const double *pose6, int K,
                       const double *w, const double *mu, const double *cov,
                       double *L_out, double *lse_out) {
    if (N <= 0 || K <= 0 || !X || !L_out) return OR_ERR_ARG;
    double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, t[3] = {0, 0, 0};
    if (pose6) { rodrigues(pose6, R); memcpy(t, pose6 + 3, sizeof(t)); }
    double *P = malloc(sizeof(double) * 9 * K), *c = malloc(sizeof(double) * K);
    if (!P || !c) { free(P); free(c); return OR_ERR_OOM; }
    int st = oracle_component_terms(K, w, cov, P, c);
    if (st != OR_OK) { free(P); free(c); return st; }
    int nt = omp_get_max_threads();
    double *Lp = calloc(nt, sizeof(double));
#pragma omp parallel
    {
        int tid = omp_get_thread_num();
        double *l = malloc(sizeof(double) * K), y[3], acc = 0.0;
#pragma omp for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            transform_point(R, t, X + 3 * n, y);
            point_logterms(y, K, mu, P, c, l);
            double v = point_lse(K, l, NULL);
            if (lse_out) lse_out[n] = v;
            acc += v;
        }
        Lp[tid] = acc;
        free(l);
    }
    double L = 0.0;
    for (int i = 0; i < nt; ++i) L += Lp[i];
    *L_out = L;
    free(Lp); free(P); free(c);
    return isfinite(L) ? OR_OK : OR_ERR_NONFINITE;
}

/* Gradient of grad_L * L(pose) with respect to the pose, the points, the
 * weights (treated as free, no renormalisation), the means and the
 * covariances (the symmetric gradient).  Any output may be NULL.
 *   d_nb      = y_n - mu_b,  Sinv_b = P_b^T P_b
 *   g_n       = dL/dy_n = -sum_b gamma_nb Sinv_b d_nb
 *   dL/dx_n   = R^T g_n,   dL/dt = sum_n g_n
 *   dL/domega = J_l(omega)^T sum_n (R x_n) x g_n
 *   dL/dmu_b  = Sinv_b sum_n gamma_nb d_nb
 *   dL/dSig_b = 1/2 Sinv_b (sum_n gamma_nb d d^T) Sinv_b - 1/2 N_b Sinv_b
 *   dL/dpi_b  = N_b / pi_b,                    N_b = sum_n gamma_nb        */
int oracle_loglik_grad(int64_t N, const double *X, const double *pose6, int K,
                       const double *w, const double *mu, const double *cov,
                       double grad_L, double *g_pose6, double *g_pts,
                       double *g_w, double *g_mu, double *g_cov) {
    if (N <= 0 || K <= 0 || !X) return OR_ERR_ARG;
    double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, t[3] = {0, 0, 0};
    double wv[3] = {0, 0, 0};
    if (pose6) {
        rodrigues(pose6, R);
        memcpy(t, pose6 + 3, sizeof(t));
        memcpy(wv, pose6, sizeof(wv));
    }
    double *P = malloc(sizeof(double) * 9 * K), *c = malloc(sizeof(double) * K);
    double *Si = malloc(sizeof(double) * 9 * K);
    if (!P || !c || !Si) { free(P); free(c); free(Si); return OR_ERR_OOM; }
    int st = oracle_component_terms(K, w, cov, P, c);
    if (st != OR_OK) { free(P); free(c); free(Si); return st; }
    for (int b = 0; b < K; ++b) {
        const double *p = P + 9 * b;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += p[k * 3 + i] * p[k * 3 + j];
                Si[9 * b + i * 3 + j] = s;
            }
    }
    int nt = omp_get_max_threads();
    /* per-thread: per component [N_b, sum g d (3), sum g d d^T (9)],
     * then [sum g_n (3), h = sum (R x) x g (3)] */
    const int per = 13;
    double *acc = calloc((size_t)nt * (K * per + 6), sizeof(double));
#pragma omp parallel
    {
        int tid = omp_get_thread_num();
        double *a = acc + (size_t)tid * (K * per + 6);
        double *l = malloc(sizeof(double) * K), *g = malloc(sizeof(double) * K);
        double y[3];
#pragma omp for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            const double *x = X + 3 * n;
            transform_point(R, t, x, y);
            point_logterms(y, K, mu, P, c, l);
            point_lse(K, l, g);
            double gn[3] = {0, 0, 0};
            for (int b = 0; b < K; ++b) {
                double d[3] = {y[0] - mu[3 * b], y[1] - mu[3 * b + 1],
                               y[2] - mu[3 * b + 2]};
                double *ab = a + per * b;
                ab[0] += g[b];
                for (int i = 0; i < 3; ++i) ab[1 + i] += g[b] * d[i];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) ab[4 + i * 3 + j] += g[b] * d[i] * d[j];
                const double *S = Si + 9 * b;
                for (int i = 0; i < 3; ++i)
                    gn[i] -= g[b] * (S[i * 3] * d[0] + S[i * 3 + 1] * d[1] + S[i * 3 + 2] * d[2]);
            }
            if (g_pts)
                for (int i = 0; i < 3; ++i)
                    g_pts[3 * n + i] = grad_L * (R[i] * gn[0] + R[3 + i] * gn[1] + R[6 + i] * gn[2]);
            double *ap = a + (size_t)K * per;
            for (int i = 0; i < 3; ++i) ap[i] += gn[i];
            double rx[3] = {y[0] - t[0], y[1] - t[1], y[2] - t[2]};
            ap[3] += rx[1] * gn[2] - rx[2] * gn[1];
            ap[4] += rx[2] * gn[0] - rx[0] * gn[2];
            ap[5] += rx[0] * gn[1] - rx[1] * gn[0];
        }
        free(l); free(g);
    }
    double *tot = calloc((size_t)K * per + 6, sizeof(double));
    for (int th = 0; th < nt; ++th)
        for (size_t i = 0; i < (size_t)K * per + 6; ++i)
            tot[i] += acc[(size_t)th * (K * per + 6) + i];
    for (int b = 0; b < K; ++b) {
        const double *ab = tot + per * b;
        const double *S = Si + 9 * b;
        if (g_w) g_w[b] = grad_L * ab[0] / w[b];
        if (g_mu)
            for (int i = 0; i < 3; ++i)
                g_mu[3 * b + i] = grad_L * (S[i * 3] * ab[1] + S[i * 3 + 1] * ab[2] + S[i * 3 + 2] * ab[3]);
        if (g_cov) {
            double T1[9], T2[9];
            matmul3(S, ab + 4, T1);
            matmul3(T1, S, T2);
            for (int i = 0; i < 9; ++i)
                g_cov[9 * b + i] = grad_L * (0.5 * T2[i] - 0.5 * ab[0] * S[i]);
        }
    }
    if (g_pose6) {
        const double *ap = tot + (size_t)K * per;
        double J[9];
        so3_left_jacobian(wv, J);
        for (int i = 0; i < 3; ++i)
            g_pose6[i] = grad_L * (J[i] * ap[3] + J[3 + i] * ap[4] + J[6 + i] * ap[5]);
        for (int i = 0; i < 3; ++i) g_pose6[3 + i] = grad_L * ap[i];
    }
    free(tot); free(acc); free(P); free(c); free(Si);
    return OR_OK;
}

/* ---- k-means++ seeding (the initialisation that precedes EM) --------------
 *
 * The paper starts EM from a responsibility matrix given by a randomised
 * k-means step (Sec. V, before "Expectation Maximization"; KInit).  The
 * reading used here is plain k-means++ D^2 seeding (Arthur & Vassilvitskii,
 * 2007) with one trial per centre and hard nearest-seed labels, no Lloyd
 * iterations.  The K random draws are inputs: u[j] in [0, 1).
 *
 *   centre 0: index floor(u[0] * N) (at most N - 1);
 *   D2_i = squared distance from x_i to the nearest centre chosen so far;
 *   centre j >= 1: with W = sum_i D2_i and t = u[j] * W, the first index
 *     whose running sum D2_0 + ... + D2_i exceeds t (so index i is drawn
 *     with probability D2_i / W); if W = 0 every point is a centre already
 *     and centre j repeats centre j - 1;
 *   label_i = index j of the nearest centre (the lowest j on ties).
 *
 * This is the definition written out: one flat running sum over the points
 * in index order, in double precision, and W is its last value.  When
 * rounding leaves no running sum above t (t within an ulp of W), the pick is
 * the last point with D2 > 0.  Squared distances are ((dx^2 + dy^2) + dz^2)
 * in double with every operation rounded on its own (the file is compiled
 * without contraction). */
static double kpp_d2(const double *a, const double *b) {
  const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return (d0 * d0 + d1 * d1) + d2 * d2;
}

/* label_i = the j whose centre X[centres[j]] is nearest to x_i, the lowest j
 * on ties (the hard assignment that turns the seeds into the first
 * responsibility matrix). */
int oracle_nearest(int64_t N, const double *X, int K, const int64_t *centres,
                   int32_t *labels) {
  if (N <= 0 || K <= 0 || !X || !centres || !labels) return OR_ERR_ARG;
  for (int j = 0; j < K; ++j)
    if (centres[j] < 0 || centres[j] >= N) return OR_ERR_ARG;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double best = kpp_d2(X + 3 * i, X + 3 * centres[0]);
    int32_t l = 0;
    for (int j = 1; j < K; ++j) {
      const double d = kpp_d2(X + 3 * i, X + 3 * centres[j]);
      if (d < best) {
        best = d;
        l = j;
      }
    }
    labels[i] = l;
  }
  return OR_OK;
}

int oracle_kmeanspp(int64_t N, const double *X, int K, const double *u,
                    int64_t *centres, int32_t *labels) {
  if (N <= 0 || K <= 0 || K > N || !X || !u || !centres) return OR_ERR_ARG;
  for (int j = 0; j < K; ++j)
    if (!(u[j] >= 0.0 && u[j] < 1.0)) return OR_ERR_ARG;
  for (int64_t i = 0; i < 3 * N; ++i)
    if (!isfinite(X[i])) return OR_ERR_NONFINITE;
  double *D = malloc((size_t)N * sizeof(double));
  if (!D) return OR_ERR_OOM;
  int64_t c0 = (int64_t)(u[0] * (double)N);
  if (c0 > N - 1) c0 = N - 1;
  centres[0] = c0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) D[i] = kpp_d2(X + 3 * i, X + 3 * c0);
  for (int j = 1; j < K; ++j) {
    double W = 0.0;
    for (int64_t i = 0; i < N; ++i) W += D[i];
    int64_t pick = centres[j - 1];
    if (W > 0.0) {
      const double t = u[j] * W;
      double acc = 0.0;
      int64_t i = 0;
      for (; i < N; ++i) {
        acc += D[i];
        if (acc > t) break;
      }
      if (i == N) {                      /* rounding: no running sum above t */
        i = N - 1;
        while (!(D[i] > 0.0)) --i;
      }
      pick = i;
    }
    centres[j] = pick;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      const double d = kpp_d2(X + 3 * i, X + 3 * pick);
      if (d < D[i]) D[i] = d;
    }
  }
  if (labels) oracle_nearest(N, X, K, centres, labels);
  free(D);
  return OR_OK;
}

/* Replay of a given seeding, for checking another implementation's picks:
 * along the centre sequence `centres` (its D2 after centres 0 .. j-1), for
 * every step j >= 1 the pick of the flat running sum above (flat_pick[j];
 * flat_pick[0] = floor(u[0] N)) and, in double-double arithmetic (Knuth's
 * error-free TwoSum, relative error of order N 2^-106), the total W and the
 * running sums before and at centres[j]: W2, before2 and at2 hold (hi, lo)
 * pairs, K x 2 each (row 0 unused). */
static void dd_add(double *hi, double *lo, double x) {
  const double s = *hi + x;
  const double bb = s - *hi;
  const double e = (*hi - (s - bb)) + (x - bb);
  const double l = *lo + e;
  const double h = s + l;
  *lo = l - (h - s);
  *hi = h;
}

int oracle_kmeanspp_replay(int64_t N, const double *X, int K, const double *u,
                           const int64_t *centres, int64_t *flat_pick,
                           double *W2, double *before2, double *at2) {
  if (N <= 0 || K <= 0 || K > N || !X || !u || !centres || !flat_pick || !W2 ||
      !before2 || !at2)
    return OR_ERR_ARG;
  for (int j = 0; j < K; ++j)
    if (centres[j] < 0 || centres[j] >= N || !(u[j] >= 0.0 && u[j] < 1.0))
      return OR_ERR_ARG;
  double *D = malloc((size_t)N * sizeof(double));
  if (!D) return OR_ERR_OOM;
  int64_t c0 = (int64_t)(u[0] * (double)N);
  if (c0 > N - 1) c0 = N - 1;
  flat_pick[0] = c0;
  for (int q = 0; q < 2; ++q) W2[q] = before2[q] = at2[q] = 0.0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) D[i] = kpp_d2(X + 3 * i, X + 3 * centres[0]);
  for (int j = 1; j < K; ++j) {
    const int64_t p = centres[j];
    double W = 0.0, wh = 0.0, wl = 0.0, bh = 0.0, bl = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      if (i == p) { bh = wh; bl = wl; }
      W += D[i];
      dd_add(&wh, &wl, D[i]);
      if (i == p) { at2[2 * j] = wh; at2[2 * j + 1] = wl; }
    }
    W2[2 * j] = wh; W2[2 * j + 1] = wl;
    before2[2 * j] = bh; before2[2 * j + 1] = bl;
    int64_t pick = centres[j - 1];
    if (W > 0.0) {
      const double t = u[j] * W;
      double acc = 0.0;
      int64_t i = 0;
      for (; i < N; ++i) {
        acc += D[i];
        if (acc > t) break;
      }
      if (i == N) {
        i = N - 1;
        while (!(D[i] > 0.0)) --i;
      }
      pick = i;
    }
    flat_pick[j] = pick;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      const double d = kpp_d2(X + 3 * i, X + 3 * p);
      if (d < D[i]) D[i] = d;
    }
  }
  free(D);
  return OR_OK;
}
