/*
 * pichol_oracle.c -- plain FP64 CPU oracle for piCholesky cross-validation.
 *
 * TEST INFRASTRUCTURE ONLY (see pichol_oracle.h).  Every loop is written in
 * the order the definition reads; OpenMP only spreads independent units
 * (rows of a Gram matrix, entries of one factor column, (fold, lambda)
 * pairs) over threads and never changes the order in which any single sum is
 * accumulated.  Built with -ffp-contract=off so that no fused multiply-add is
 * formed behind the reader's back.
 *
 * Section numbers refer to Kuang, Gittens, Hamid (arXiv 1404.0466).
 */
#include "pichol_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int32_t orc_num_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int32_t n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads((int)n);
#else
  (void)n;
#endif
}

/* numpy.array_split sizes: the first n % k folds get one extra row. */
void orc_fold_bounds(int64_t n, int32_t k, int64_t *start) {
  int64_t base = n / k, extra = n % k;
  start[0] = 0;
  for (int32_t f = 0; f < k; ++f)
    start[f + 1] = start[f] + base + (f < extra ? 1 : 0);
}

/* Sec. 3.1: H = X^T X and g = X^T y over the training rows of fold f.  Each
 * entry is a sum over training rows in increasing row order. */
int64_t orc_fold_gram(int64_t n, int64_t d, int64_t c, int32_t k, int32_t f,
                      const double *X, const double *Y, int normalize,
                      double *H, double *B) {
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k + 1));
  orc_fold_bounds(n, k, start);
  int64_t v0 = start[f], v1 = start[f + 1];
  free(start);
  int64_t ntr = n - (v1 - v0);
  double scale = normalize ? 1.0 / (double)ntr : 1.0;

#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < d; ++i) {
    double *hrow = H + i * d;
    double *brow = B + i * c;
    for (int64_t j = 0; j <= i; ++j) hrow[j] = 0.0;
    for (int64_t cc = 0; cc < c; ++cc) brow[cc] = 0.0;
    for (int64_t row = 0; row < n; ++row) {
      if (row >= v0 && row < v1) continue; /* validation row */
      const double *x = X + row * d;
      const double *y = Y + row * c;
      double xi = x[i];
      for (int64_t j = 0; j <= i; ++j) hrow[j] += xi * x[j];
      for (int64_t cc = 0; cc < c; ++cc) brow[cc] += xi * y[cc];
    }
    for (int64_t j = 0; j <= i; ++j) hrow[j] *= scale;
    for (int64_t cc = 0; cc < c; ++cc) brow[cc] *= scale;
  }
  /* mirror into the upper triangle */
  for (int64_t i = 0; i < d; ++i)
    for (int64_t j = i + 1; j < d; ++j) H[i * d + j] = H[j * d + i];
  return ntr;
}

/* Sec. 3.2: A + lam I = L L^T.  Column j: the diagonal entry is the square
 * root of what is left of A_jj after removing the contributions of the
 * earlier columns, and every entry below it is what is left of A_ij divided
 * by that diagonal. */
int32_t orc_cholesky(int64_t d, const double *A, double lam, double *L) {
  memset(L, 0, sizeof(double) * (size_t)(d * d));
  for (int64_t j = 0; j < d; ++j) {
    const double *lj = L + j * d;
    double s = A[j * d + j] + lam;
    for (int64_t p = 0; p < j; ++p) s -= lj[p] * lj[p];
    if (!(s > 0.0)) return (int32_t)(j + 1);
    double ljj = sqrt(s);
    L[j * d + j] = ljj;
#pragma omp parallel for schedule(static) if (d - j > 256)
    for (int64_t i = j + 1; i < d; ++i) {
      const double *li = L + i * d;
      double t = A[i * d + j];
      for (int64_t p = 0; p < j; ++p) t -= li[p] * lj[p];
      L[i * d + j] = t / ljj;
    }
  }
  return 0;
}

void orc_pack_lower(int64_t d, const double *L, double *t) {
  int64_t e = 0;
  for (int64_t i = 0; i < d; ++i)
    for (int64_t j = 0; j <= i; ++j) t[e++] = L[i * d + j];
}

void orc_unpack_lower(int64_t d, const double *t, double *L) {
  memset(L, 0, sizeof(double) * (size_t)(d * d));
  int64_t e = 0;
  for (int64_t i = 0; i < d; ++i)
    for (int64_t j = 0; j <= i; ++j) L[i * d + j] = t[e++];
}

/* Algorithm 1, steps 3-6 (Sec. 3.3).  The monomial basis is taken in
 * tau = lam / lam_ref: the same polynomial space as monomials in lam, related
 * by the diagonal change of basis diag(lam_ref^-j) (Sec. 4, proof of the
 * stability theorem), chosen so that V stays well conditioned when the
 * sample values are small. */
/* The variable of the fitted polynomials: tau = lam / lam_ref (basis 0, the
 * paper's polynomials in lambda) or u = log(lam / lam_ref) (basis 1,
 * polynomials in log lambda). */
static double basis_var(double lam, double lam_ref, int32_t basis) {
  return basis ? log(lam / lam_ref) : lam / lam_ref;
}

int32_t orc_fit(int64_t D, int32_t g, int32_t r, const double *lam_s,
                double lam_ref, const double *T, double *Theta,
                int32_t basis) {
  if (r < 0 || r > 63 || g <= r || !(lam_ref > 0.0)) return -1;
  int32_t m = r + 1;
  double *V = (double *)malloc(sizeof(double) * (size_t)(g * m));
  double *Hl = (double *)malloc(sizeof(double) * (size_t)(m * m));
  double *Rl = (double *)malloc(sizeof(double) * (size_t)(m * m));
  /* step 3-4: leftmost r+1 columns of the g x g Vandermonde matrix */
  for (int32_t s = 0; s < g; ++s) {
    double tau = basis_var(lam_s[s], lam_ref, basis), p = 1.0;
    for (int32_t j = 0; j < m; ++j) {
      V[s * m + j] = p;
      p *= tau;
    }
  }
  /* step 5: H_l = V^T V */
  for (int32_t a = 0; a < m; ++a)
    for (int32_t b = 0; b < m; ++b) {
      double acc = 0.0;
      for (int32_t s = 0; s < g; ++s) acc += V[s * m + a] * V[s * m + b];
      Hl[a * m + b] = acc;
    }
  /* H_l is symmetric positive definite when the samples are distinct:
   * factor it to apply H_l^{-1}. */
  if (orc_cholesky(m, Hl, 0.0, Rl) != 0) {
    free(V);
    free(Hl);
    free(Rl);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < D; ++e) {
    double Gcol[64], z[64];
    /* step 5: column e of G_l = V^T T */
    for (int32_t a = 0; a < m; ++a) {
      double acc = 0.0;
      for (int32_t s = 0; s < g; ++s) acc += V[s * m + a] * T[(int64_t)s * D + e];
      Gcol[a] = acc;
    }
    /* step 6: Theta column = H_l^{-1} G column, via R R^T x = G */
    for (int32_t a = 0; a < m; ++a) {
      double acc = Gcol[a];
      for (int32_t b = 0; b < a; ++b) acc -= Rl[a * m + b] * z[b];
      z[a] = acc / Rl[a * m + a];
    }
    for (int32_t a = m - 1; a >= 0; --a) {
      double acc = z[a];
      for (int32_t b = a + 1; b < m; ++b) acc -= Rl[b * m + a] * Theta[(int64_t)b * D + e];
      Theta[(int64_t)a * D + e] = acc / Rl[a * m + a];
    }
  }
  free(V);
  free(Hl);
  free(Rl);
  return 0;
}

/* Sec. 3.3: the interpolated factor at a new lambda is every fitted
 * polynomial evaluated there. */
void orc_eval(int64_t D, int32_t r, const double *Theta, double lam,
              double lam_ref, double *out, int32_t basis) {
  double tau = basis_var(lam, lam_ref, basis);
  for (int64_t e = 0; e < D; ++e) {
    double acc = 0.0, p = 1.0;
    for (int32_t j = 0; j <= r; ++j) {
      acc += p * Theta[(int64_t)j * D + e];
      p *= tau;
    }
    out[e] = acc;
  }
}

void orc_eval_deriv(int64_t D, int32_t r, const double *Theta, double lam,
                    double lam_ref, double *out, int32_t basis) {
  double tau = basis_var(lam, lam_ref, basis);
  /* d(var)/d(lam): 1/lam_ref for tau, 1/lam for log(lam/lam_ref) */
  double dvar = basis ? 1.0 / lam : 1.0 / lam_ref;
  for (int64_t e = 0; e < D; ++e) {
    double acc = 0.0, p = 1.0; /* p = tau^(j-1) */
    for (int32_t j = 1; j <= r; ++j) {
      acc += (double)j * p * Theta[(int64_t)j * D + e];
      p *= tau;
    }
    out[e] = acc * dvar;
  }
}

/* Sec. 3.2: L w = g by forward substitution, then L^T theta = w by back
 * substitution, for each of the c columns. */
int32_t orc_solve(int64_t d, int64_t c, const double *L, const double *B,
                  double *W) {
  int32_t flags = 0;
  for (int64_t i = 0; i < d; ++i)
    if (!(L[i * d + i] > 0.0)) flags |= 2;
  double *U = (double *)malloc(sizeof(double) * (size_t)(d * c));
  for (int64_t cc = 0; cc < c; ++cc) {
    for (int64_t i = 0; i < d; ++i) { /* forward, rows ascending */
      double acc = B[i * c + cc];
      for (int64_t p = 0; p < i; ++p) acc -= L[i * d + p] * U[p * c + cc];
      U[i * c + cc] = acc / L[i * d + i];
    }
    for (int64_t i = d - 1; i >= 0; --i) { /* back, rows descending */
      double acc = U[i * c + cc];
      for (int64_t p = i + 1; p < d; ++p) acc -= L[p * d + i] * W[p * c + cc];
      W[i * c + cc] = acc / L[i * d + i];
    }
  }
  free(U);
  for (int64_t e = 0; e < d * c; ++e)
    if (!isfinite(W[e])) {
      flags |= 1;
      break;
    }
  return flags;
}

int32_t orc_refine(int64_t d, int64_t c, const double *H, double lam,
                   const double *L, const double *B, double *W,
                   int32_t steps) {
  int32_t flags = 0;
  double *R = (double *)malloc(sizeof(double) * (size_t)(d * c));
  double *D = (double *)malloc(sizeof(double) * (size_t)(d * c));
  for (int32_t it = 0; it < steps; ++it) {
    for (int64_t i = 0; i < d; ++i)
      for (int64_t cc = 0; cc < c; ++cc) {
        double acc = 0.0; /* ((H + lam I) W)_{i,cc} */
        for (int64_t p = 0; p < d; ++p) acc += H[i * d + p] * W[p * c + cc];
        acc += lam * W[i * c + cc];
        R[i * c + cc] = B[i * c + cc] - acc;
      }
    flags |= orc_solve(d, c, L, R, D);
    for (int64_t e = 0; e < d * c; ++e) W[e] += D[e];
  }
  free(R);
  free(D);
  return flags;
}

/* Hold-out residual R = Y_v - X_v W and its sum of squares. */
double orc_holdout_sse(int64_t nv, int64_t d, int64_t c, const double *Xv,
                       int64_t ldx, const double *Yv, int64_t ldy,
                       const double *W) {
  double sse = 0.0;
  for (int64_t row = 0; row < nv; ++row) {
    const double *x = Xv + row * ldx;
    for (int64_t cc = 0; cc < c; ++cc) {
      double pred = 0.0;
      for (int64_t p = 0; p < d; ++p) pred += x[p] * W[p * c + cc];
      double res = Yv[row * ldy + cc] - pred;
      sse += res * res;
    }
  }
  return sse;
}

double orc_holdout_sst(int64_t nv, int64_t c, const double *Yv, int64_t ldy) {
  double sst = 0.0;
  for (int64_t cc = 0; cc < c; ++cc) {
    double mean = 0.0;
    for (int64_t row = 0; row < nv; ++row) mean += Yv[row * ldy + cc];
    mean /= (double)nv;
    for (int64_t row = 0; row < nv; ++row) {
      double dv = Yv[row * ldy + cc] - mean;
      sst += dv * dv;
    }
  }
  return sst;
}

/* Normalised root-mean-squared error of a fitted factor (the accuracy
 * measure of the paper's NRMSE section): over the d(d+1)/2 entries with
 * i >= j of dense row-major d x d lower factors,
 *   sqrt(sum (Lhat - L)^2) / sqrt(sum (L - mean L)^2),
 * the mean taken over those entries (two passes, rows then columns in
 * increasing order).  Predicting every entry by the mean gives 1. */
double orc_factor_nrmse(int64_t d, const double *Lhat, const double *L) {
  double sum = 0.0;
  int64_t cnt = 0;
  for (int64_t i = 0; i < d; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      sum += L[i * d + j];
      ++cnt;
    }
  const double mean = sum / (double)cnt;
  double sd = 0.0, ss = 0.0;
  for (int64_t i = 0; i < d; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      const double e = Lhat[i * d + j] - L[i * d + j];
      const double v = L[i * d + j] - mean;
      sd += e * e;
      ss += v * v;
    }
  return sqrt(sd) / sqrt(ss);
}

/* One (fold, lambda) unit downstream of a factor: solve (then `refine`
 * steps of refinement against H + lam I), then hold-out. */
static void unit_solve_holdout(int64_t d, int64_t c, const double *L,
                               const double *B, const double *H, double lam,
                               int32_t refine, int64_t nv, const double *Xv,
                               int64_t ldx, const double *Yv, int64_t ldy,
                               double *Wout, double *mse, double *sse,
                               int32_t *flags) {
  double *W = Wout ? Wout : (double *)malloc(sizeof(double) * (size_t)(d * c));
  int32_t fl = orc_solve(d, c, L, B, W);
  if (refine > 0) fl |= orc_refine(d, c, H, lam, L, B, W, refine);
  double s = orc_holdout_sse(nv, d, c, Xv, ldx, Yv, ldy, W);
  if (!isfinite(s)) fl |= 1;
  *flags = fl;
  if (sse) *sse = s;
  *mse = s / ((double)nv * (double)c);
  if (!Wout) free(W);
}

int32_t orc_cv_exact(int64_t n, int64_t d, int64_t c, int32_t k, int32_t q,
                     int normalize, const double *X, const double *Y,
                     const double *lam_grid, double *mse, double *sse,
                     double *W, int32_t *info, int32_t *flags,
                     int32_t refine) {
  if (n < k || k < 2 || d < 1 || c < 1 || q < 1 || refine < 0) return -1;
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k + 1));
  orc_fold_bounds(n, k, start);
  double *H = (double *)malloc(sizeof(double) * (size_t)(d * d));
  double *B = (double *)malloc(sizeof(double) * (size_t)(d * c));
  for (int32_t f = 0; f < k; ++f) {
    orc_fold_gram(n, d, c, k, f, X, Y, normalize, H, B);
    int64_t nv = start[f + 1] - start[f];
    const double *Xv = X + start[f] * d, *Yv = Y + start[f] * c;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < q; ++t) {
      double *L = (double *)malloc(sizeof(double) * (size_t)(d * d));
      int64_t u = (int64_t)f * q + t;
      info[u] = orc_cholesky(d, H, lam_grid[t], L);
      double *Wt = W ? W + u * d * c : NULL;
      if (info[u] != 0) {
        /* the factorization does not exist: report NaN, like the solve of a
         * failed factor would */
        for (int64_t e = 0; Wt && e < d * c; ++e) Wt[e] = NAN;
        mse[u] = NAN;
        if (sse) sse[u] = NAN;
        flags[u] = 1;
      } else {
        unit_solve_holdout(d, c, L, B, H, lam_grid[t], refine, nv, Xv, d, Yv,
                           c, Wt, &mse[u], sse ? &sse[u] : NULL, &flags[u]);
      }
      free(L);
    }
  }
  free(H);
  free(B);
  free(start);
  return 0;
}

int32_t orc_fold_interp(int64_t d, int64_t c, int32_t g, int32_t r, int32_t q,
                        const double *H, const double *B, int64_t nv,
                        const double *Xv, int64_t ldx, const double *Yv,
                        int64_t ldy, const double *lam_s,
                        const double *lam_grid, double lam_ref, double *mse,
                        double *W, int32_t *info, int32_t *flags,
                        int32_t refine, int32_t basis) {
  if (refine < 0) return -1;
  int64_t D = d * (d + 1) / 2;
  double *T = (double *)malloc(sizeof(double) * (size_t)(g * D));
  double *Theta = (double *)malloc(sizeof(double) * (size_t)((r + 1) * D));
  /* Algorithm 1 step 1-2: exact factors at the sample values, vectorised
   * into the rows of T */
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t s = 0; s < g; ++s) {
    double *L = (double *)malloc(sizeof(double) * (size_t)(d * d));
    info[s] = orc_cholesky(d, H, lam_s[s], L);
    if (info[s] != 0)
      for (int64_t e = 0; e < d * d; ++e) L[e] = NAN;
    orc_pack_lower(d, L, T + (int64_t)s * D);
    free(L);
  }
  int32_t rc = orc_fit(D, g, r, lam_s, lam_ref, T, Theta, basis);
  free(T);
  if (rc != 0) {
    free(Theta);
    return rc;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t t = 0; t < q; ++t) {
    double *lt = (double *)malloc(sizeof(double) * (size_t)D);
    double *L = (double *)malloc(sizeof(double) * (size_t)(d * d));
    orc_eval(D, r, Theta, lam_grid[t], lam_ref, lt, basis);
    orc_unpack_lower(d, lt, L);
    unit_solve_holdout(d, c, L, B, H, lam_grid[t], refine, nv, Xv, ldx, Yv,
                       ldy, W ? W + (int64_t)t * d * c : NULL, &mse[t], NULL,
                       &flags[t]);
    free(L);
    free(lt);
  }
  free(Theta);
  return 0;
}

int32_t orc_cv_interp(int64_t n, int64_t d, int64_t c, int32_t k, int32_t g,
                      int32_t r, int32_t q, int normalize, const double *X,
                      const double *Y, const double *lam_s,
                      const double *lam_grid, double lam_ref, double *mse,
                      double *sse, double *W, double *Theta_out, int32_t *info,
                      int32_t *flags, int32_t refine, int32_t basis) {
  if (n < k || k < 2 || d < 1 || c < 1 || q < 1 || r < 0 || g <= r ||
      !(lam_ref > 0.0) || refine < 0)
    return -1;
  int64_t D = d * (d + 1) / 2;
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k + 1));
  orc_fold_bounds(n, k, start);
  double *H = (double *)malloc(sizeof(double) * (size_t)(d * d));
  double *B = (double *)malloc(sizeof(double) * (size_t)(d * c));
  double *T = (double *)malloc(sizeof(double) * (size_t)(g * D));
  double *Theta = (double *)malloc(sizeof(double) * (size_t)((r + 1) * D));
  int32_t rc = 0;
  for (int32_t f = 0; f < k && rc == 0; ++f) {
    orc_fold_gram(n, d, c, k, f, X, Y, normalize, H, B);
    int64_t nv = start[f + 1] - start[f];
    const double *Xv = X + start[f] * d, *Yv = Y + start[f] * c;
    /* Algorithm 1 step 1-2 */
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t s = 0; s < g; ++s) {
      double *L = (double *)malloc(sizeof(double) * (size_t)(d * d));
      info[(int64_t)f * g + s] = orc_cholesky(d, H, lam_s[s], L);
      if (info[(int64_t)f * g + s] != 0)
        for (int64_t e = 0; e < d * d; ++e) L[e] = NAN;
      orc_pack_lower(d, L, T + (int64_t)s * D);
      free(L);
    }
    /* Algorithm 1 step 3-6 */
    rc = orc_fit(D, g, r, lam_s, lam_ref, T, Theta, basis);
    if (rc != 0) break;
    if (Theta_out)
      memcpy(Theta_out + (int64_t)f * (r + 1) * D, Theta,
             sizeof(double) * (size_t)((r + 1) * D));
    /* evaluation at every grid value, then the exact method's solves */
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < q; ++t) {
      int64_t u = (int64_t)f * q + t;
      double *lt = (double *)malloc(sizeof(double) * (size_t)D);
      double *L = (double *)malloc(sizeof(double) * (size_t)(d * d));
      orc_eval(D, r, Theta, lam_grid[t], lam_ref, lt, basis);
      orc_unpack_lower(d, lt, L);
      unit_solve_holdout(d, c, L, B, H, lam_grid[t], refine, nv, Xv, d, Yv,
                         c, W ? W + u * d * c : NULL, &mse[u],
                         sse ? &sse[u] : NULL, &flags[u]);
      free(L);
      free(lt);
    }
  }
  free(H);
  free(B);
  free(T);
  free(Theta);
  free(start);
  return rc;
}

/* out = M^T x for a dense lower d x d M (row-major) and x d x c. */
static void lower_t_times(int64_t d, int64_t c, const double *M,
                          const double *x, double *out) {
  for (int64_t i = 0; i < d; ++i)
    for (int64_t cc = 0; cc < c; ++cc) {
      double acc = 0.0;
      for (int64_t p = i; p < d; ++p) acc += M[p * d + i] * x[p * c + cc];
      out[i * c + cc] = acc;
    }
}

/* One (fold, lambda) of the gradient, given the factor L of A and, for
 * piCholesky, dL = dLhat/dlambda (NULL for the exact method, dA = I). */
static void unit_grad(int64_t d, int64_t c, const double *L, const double *dL,
                      const double *B, int64_t nv, const double *Xv,
                      const double *Yv, double lam, double *mse, double *dlog,
                      int32_t *flags) {
  size_t dc = (size_t)(d * c);
  double *th = (double *)malloc(sizeof(double) * dc);
  double *s = (double *)malloc(sizeof(double) * dc);
  double *z = (double *)malloc(sizeof(double) * dc);
  int32_t fl = orc_solve(d, c, L, B, th);
  /* s = X_v^T R, R = Y_v - X_v theta, row by row */
  for (size_t e = 0; e < dc; ++e) s[e] = 0.0;
  double sse = 0.0;
  for (int64_t row = 0; row < nv; ++row) {
    const double *x = Xv + row * d;
    for (int64_t cc = 0; cc < c; ++cc) {
      double pred = 0.0;
      for (int64_t p = 0; p < d; ++p) pred += x[p] * th[p * c + cc];
      double res = Yv[row * c + cc] - pred;
      sse += res * res;
      for (int64_t p = 0; p < d; ++p) s[p * c + cc] += x[p] * res;
    }
  }
  fl |= orc_solve(d, c, L, s, z);
  double dot = 0.0;
  if (dL) {
    double *a1 = (double *)malloc(sizeof(double) * dc); /* Lhat^T theta */
    double *b1 = (double *)malloc(sizeof(double) * dc); /* dLhat^T theta */
    double *a2 = (double *)malloc(sizeof(double) * dc); /* Lhat^T z */
    double *b2 = (double *)malloc(sizeof(double) * dc); /* dLhat^T z */
    lower_t_times(d, c, L, th, a1);
    lower_t_times(d, c, dL, th, b1);
    lower_t_times(d, c, L, z, a2);
    lower_t_times(d, c, dL, z, b2);
    for (size_t e = 0; e < dc; ++e) dot += b2[e] * a1[e] + a2[e] * b1[e];
    free(a1);
    free(b1);
    free(a2);
    free(b2);
  } else {
    for (size_t e = 0; e < dc; ++e) dot += z[e] * th[e];
  }
  double cnt = (double)nv * (double)c;
  *mse = sse / cnt;
  *dlog = lam * 2.0 * dot / cnt;
  if (!isfinite(*mse) || !isfinite(*dlog)) fl |= 1;
  *flags = fl;
  free(th);
  free(s);
  free(z);
}

int32_t orc_cv_grad(int64_t n, int64_t d, int64_t c, int32_t k, int32_t g,
                    int32_t r, int32_t q, int normalize, int interp,
                    const double *X, const double *Y, const double *lam_s,
                    const double *lam_grid, double lam_ref, double *mse,
                    double *dlog, int32_t *info, int32_t *flags,
                    int32_t basis) {
  if (n < k || k < 2 || d < 1 || c < 1 || q < 1) return -1;
  if (interp && (r < 0 || g <= r || !(lam_ref > 0.0))) return -1;
  int64_t D = d * (d + 1) / 2;
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k + 1));
  orc_fold_bounds(n, k, start);
  double *H = (double *)malloc(sizeof(double) * (size_t)(d * d));
  double *B = (double *)malloc(sizeof(double) * (size_t)(d * c));
  double *T = interp ? (double *)malloc(sizeof(double) * (size_t)(g * D)) : NULL;
  double *Theta =
      interp ? (double *)malloc(sizeof(double) * (size_t)((r + 1) * D)) : NULL;
  int32_t rc = 0;
  for (int32_t f = 0; f < k && rc == 0; ++f) {
    orc_fold_gram(n, d, c, k, f, X, Y, normalize, H, B);
    int64_t nv = start[f + 1] - start[f];
    const double *Xv = X + start[f] * d, *Yv = Y + start[f] * c;
    if (interp) {
#pragma omp parallel for schedule(dynamic, 1)
      for (int32_t s = 0; s < g; ++s) {
        double *L = (double *)malloc(sizeof(double) * (size_t)(d * d));
        info[(int64_t)f * g + s] = orc_cholesky(d, H, lam_s[s], L);
        if (info[(int64_t)f * g + s] != 0)
          for (int64_t e = 0; e < d * d; ++e) L[e] = NAN;
        orc_pack_lower(d, L, T + (int64_t)s * D);
        free(L);
      }
      rc = orc_fit(D, g, r, lam_s, lam_ref, T, Theta, basis);
      if (rc != 0) break;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < q; ++t) {
      int64_t u = (int64_t)f * q + t;
      double *L = (double *)malloc(sizeof(double) * (size_t)(d * d));
      double *dL = NULL;
      if (interp) {
        double *lt = (double *)malloc(sizeof(double) * (size_t)D);
        dL = (double *)malloc(sizeof(double) * (size_t)(d * d));
        orc_eval(D, r, Theta, lam_grid[t], lam_ref, lt, basis);
        orc_unpack_lower(d, lt, L);
        orc_eval_deriv(D, r, Theta, lam_grid[t], lam_ref, lt, basis);
        orc_unpack_lower(d, lt, dL);
        free(lt);
      } else {
        info[u] = orc_cholesky(d, H, lam_grid[t], L);
      }
      if (!interp && info[u] != 0) {
        mse[u] = NAN;
        dlog[u] = NAN;
        flags[u] = 1;
      } else {
        unit_grad(d, c, L, dL, B, nv, Xv, Yv, lam_grid[t], &mse[u], &dlog[u],
                  &flags[u]);
      }
      free(L);
      free(dL);
    }
  }
  free(H);
  free(B);
  free(T);
  free(Theta);
  free(start);
  return rc;
}

