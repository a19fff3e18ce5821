/*
 * pichol_oracle.h -- plain FP64 CPU oracle for piCholesky cross-validation.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * Paper: Kuang, Gittens, Hamid, "Cholesky Factor Interpolation for Efficient
 * Approximate Cross-Validation" (arXiv 1404.0466).
 *
 * Conventions (all arrays row-major, FP64, host memory, caller-owned):
 *   X      n x d   design matrix (no intercept column is added here; a caller
 *                  that wants the paper's intercept appends a column of ones)
 *   Y      n x c   right-hand sides (label columns)
 *   folds  contiguous, sizes as numpy.array_split(range(n), k): the first
 *          n mod k folds hold one extra row
 *   H_f    d x d   X_tr^T X_tr (divided by n_tr when normalize != 0)
 *   B_f    d x c   X_tr^T Y_tr (same scaling)
 *   packed triangle vector: entry (i,j), j <= i, sits at i(i+1)/2 + j
 *
 * Status / flag conventions (shared in meaning, not in code, with the GPU
 * library):
 *   info  = 0 when the factorization succeeded, j+1 when the pivot of
 *           column j (0-based) was not positive (LAPACK convention)
 *   flags bit0 = some solution or hold-out value is not finite
 *         bit1 = some diagonal entry of the (interpolated) factor is <= 0
 */
#ifndef PICHOL_ORACLE_H
#define PICHOL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Fold f owns rows [start[f], start[f+1]) with start[0]=0, start[k]=n. */
void orc_fold_bounds(int64_t n, int32_t k, int64_t *start);

/* Gram matrices of one training fold (Sec. 3.1, regularised normal
 * equations): H = X_tr^T X_tr, B = X_tr^T Y_tr, summed over training rows in
 * increasing row order, divided by n_tr when normalize != 0.  H is written in
 * full (both triangles).  Returns n_tr. */
int64_t orc_fold_gram(int64_t n, int64_t d, int64_t c, int32_t k, int32_t f,
                      const double *X, const double *Y, int normalize,
                      double *H, double *B);

/* Cholesky factor of A + lam*I (Sec. 3.2), column by column (Crout order).
 * Reads the lower triangle of A (d x d).  Writes the full d x d L with zeros
 * above the diagonal.  Returns info (0 or first failing column + 1). */
int32_t orc_cholesky(int64_t d, const double *A, double lam, double *L);

/* Vectorise the lower triangle of L (d x d) row-wise into t[D]. */
void orc_pack_lower(int64_t d, const double *L, double *t);
/* Inverse of orc_pack_lower; zeros above the diagonal. */
void orc_unpack_lower(int64_t d, const double *t, double *L);

/* Algorithm 1, steps 3-6 (Sec. 3.3): observation matrix V (g x (r+1)) of
 * monomials in tau = lam/lam_ref at the g sample values, H_l = V^T V,
 * G_l = V^T T, Theta = H_l^{-1} G_l.  T is g x D, Theta is (r+1) x D.
 * Returns 0, or -1 when the arguments are invalid (r >= g, lam_ref <= 0) or
 * H_l is singular (repeated sample values). */
int32_t orc_fit(int64_t D, int32_t g, int32_t r, const double *lam_s,
                double lam_ref, const double *T, double *Theta,
                int32_t basis);

/* Evaluate the D fitted polynomials at lam (Sec. 3.3): out[e] =
 * sum_j (lam/lam_ref)^j Theta[j][e]. */
void orc_eval(int64_t D, int32_t r, const double *Theta, double lam,
              double lam_ref, double *out,
              int32_t basis);

/* Basis of the fitted polynomials (the last argument of the fit, evaluation
 * and interpolated-CV functions): 0 = monomials in tau = lam / lam_ref, the
 * polynomial space of Algorithm 1 (polynomials in lambda); 1 = monomials in
 * u = log(lam / lam_ref), polynomials in log lambda (all lambdas > 0). */

/* Derivative of the interpolated factor with respect to lambda:
 * sum_j j tau^(j-1) / lam_ref Theta_j, tau = lam / lam_ref. */
void orc_eval_deriv(int64_t D, int32_t r, const double *Theta, double lam,
                    double lam_ref, double *out,
                    int32_t basis);

/* Forward substitution L U = B, then back substitution L^T W = U
 * (Sec. 3.2).  L is d x d lower (only the lower triangle is read), B and W are
 * d x c.  Never aborts.  Returns flag bits (bit1: some L_ii <= 0, bit0: some
 * W entry not finite). */
int32_t orc_solve(int64_t d, int64_t c, const double *L, const double *B,
                  double *W);

/* Hold-out residual sum of squares: R = Y_v - X_v W, returns sum(R^2).  Xv
 * has leading dimension ldx, Yv leading dimension ldy. */
double orc_holdout_sse(int64_t nv, int64_t d, int64_t c, const double *Xv,
                       int64_t ldx, const double *Yv, int64_t ldy,
                       const double *W);

/* Sum over the c columns of the squared deviation of Y_v from its column
 * means (the denominator of the normalised RMSE). */
double orc_holdout_sst(int64_t nv, int64_t c, const double *Yv, int64_t ldy);
/* sqrt(sum (Lhat - L)^2) / sqrt(sum (L - mean L)^2) over the entries i >= j
 * of dense row-major d x d lower factors (NRMSE section). */
double orc_factor_nrmse(int64_t d, const double *Lhat, const double *L);

/* Iterative refinement of the solution of (H + lam I) W = B (the classic
 * residual-correction method, e.g. Higham, "Accuracy and Stability of
 * Numerical Algorithms", ch. 12), reusing the factor L of the first solve:
 * `steps` times, R = B - (H + lam I) W (FP64, row by row, terms in
 * increasing column order), then W += the solution of L L^T D = R
 * (orc_solve).  H: d x d symmetric (both triangles); L: d x d lower;
 * B, W: d x c.  With an exact factor the corrections are rounding-sized;
 * with an approximate one (an interpolated factor, a lower-precision one)
 * W converges to (H + lam I)^{-1} B when the spectral radius of
 * I - (L L^T)^{-1}(H + lam I) is below one.  Returns orc_solve's flags
 * OR-ed over the correction solves. */
int32_t orc_refine(int64_t d, int64_t c, const double *H, double lam,
                   const double *L, const double *B, double *W,
                   int32_t steps);

/* Whole k-fold cross-validation, exact Cholesky at every grid value
 * (Sec. 3.2 and the exact baseline of Sec. 6.2).
 *   mse   k x q   sum(R^2)/(n_v c)
 *   sse   k x q   sum(R^2)                      (may be NULL)
 *   W     k x q x d x c solutions               (may be NULL)
 *   info  k x q
 *   flags k x q
 * refine >= 0 steps of orc_refine follow every solve.
 * Returns 0, or -1 on invalid arguments. */
int32_t orc_cv_exact(int64_t n, int64_t d, int64_t c, int32_t k, int32_t q,
                     int normalize, const double *X, const double *Y,
                     const double *lam_grid, double *mse, double *sse,
                     double *W, int32_t *info, int32_t *flags,
                     int32_t refine);

/* Whole k-fold cross-validation with piCholesky (Algorithm 1 followed by
 * evaluation at every grid value and the same solves):
 *   info  k x g (one per sample factorization)
 *   flags k x q
 * Theta (k x (r+1) x D, may be NULL) receives the fitted coefficients.
 * refine >= 0 steps of orc_refine against H_f + lambda_t I follow every
 * solve, with the interpolated factor as the preconditioner. */
int32_t orc_cv_interp(int64_t n, int64_t d, int64_t c, int32_t k, int32_t g,
                      int32_t r, int32_t q, int normalize, const double *X,
                      const double *Y, const double *lam_s,
                      const double *lam_grid, double lam_ref, double *mse,
                      double *sse, double *W, double *Theta, int32_t *info,
                      int32_t *flags, int32_t refine,
                      int32_t basis);

/* The per-fold part of orc_cv_interp starting from that fold's H_f, B_f and
 * validation rows (used to time one fold without the Gram step).
 * mse, W (may be NULL), flags have q entries / q x d x c; info has g. */
int32_t orc_fold_interp(int64_t d, int64_t c, int32_t g, int32_t r, int32_t q,
                        const double *H, const double *B, int64_t nv,
                        const double *Xv, int64_t ldx, const double *Yv,
                        int64_t ldy, const double *lam_s,
                        const double *lam_grid, double lam_ref, double *mse,
                        double *W, int32_t *info, int32_t *flags,
                        int32_t refine,
                      int32_t basis);

/* Derivative of the hold-out error with respect to log lambda, for every
 * fold and grid value (the differentiation form).  With A the matrix whose
 * Cholesky factor the method uses at lambda (Lhat Lhat^T for piCholesky,
 * H_f + lambda I for the exact method), theta = A^{-1} B_f,
 * R = Y_v - X_v theta and z = A^{-1} X_v^T R:
 *   d mse / d lambda = 2/(n_v c) <z, (dA/dlambda) theta>,
 * with dA = dLhat Lhat^T + Lhat dLhat^T and dLhat = orc_eval_deriv for
 * piCholesky, so the product is <dLhat^T z, Lhat^T theta> +
 * <Lhat^T z, dLhat^T theta>; dA = I for the exact method.
 * dlog = lambda * d mse / d lambda.  mse as in the CV calls.
 * interp != 0: piCholesky (lam_s, r used); interp == 0: exact factors.
 * Returns 0, or -1 on invalid arguments. */
int32_t orc_cv_grad(int64_t n, int64_t d, int64_t c, int32_t k, int32_t g,
                    int32_t r, int32_t q, int normalize, int interp,
                    const double *X, const double *Y, const double *lam_s,
                    const double *lam_grid, double lam_ref, double *mse,
                    double *dlog, int32_t *info, int32_t *flags,
                      int32_t basis);

/* Number of OpenMP threads the oracle runs with. */
int32_t orc_num_threads(void);
/* Threads of the OpenMP regions that follow (n >= 1; no arithmetic). */
void orc_set_num_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
