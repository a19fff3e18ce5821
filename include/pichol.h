/*
 * pichol.h -- C-ABI of the MI355X (gfx950) piCholesky cross-validation
 * library.
 *
 * Method: Kuang, Gittens, Hamid, "Cholesky Factor Interpolation for
 * Efficient Approximate Cross-Validation" (arXiv 1404.0466).  Ridge
 * regression theta = (H + lambda I)^{-1} g with H = X^T X, g = X^T y
 * (Sec. 3.1, regularised normal equations), solved through a Cholesky factor
 * and two triangular solves (Sec. 3.2).  piCholesky (Algorithm 1, Sec. 3.3)
 * factors H + lambda_s I exactly at g sample values, fits a polynomial of
 * degree r in lambda to every entry of the factor by least squares, and
 * evaluates the polynomials at the dense grid instead of factoring there.
 *
 * General conventions
 * -------------------
 *  - Every pointer documented "device" is HIP device memory owned by the
 *    caller; "host" pointers are read before the call returns.  The library
 *    allocates no memory: scratch space comes from the caller's workspace.
 *  - Work is enqueued on the caller's stream; calls return after enqueueing.
 *    Inputs must stay valid until the stream reaches the end of the work.
 *  - Argument errors are returned synchronously before anything is
 *    enqueued.  Data errors are reported asynchronously in device arrays:
 *      info[u]  = 0, or j+1 when the pivot of column j (0-based) of a shifted
 *                 matrix was not positive (LAPACK convention); the outputs
 *                 that depend on that factor are then NaN;
 *      flags[u] bit0 = a solution or hold-out error is not finite,
 *               bit1 = a diagonal entry of an interpolated factor is <= 0
 *                      (and, in pichol_solve_factors, of a given factor;
 *                      the cross-validation calls report a failed exact
 *                      factorization through info, and its NaN results
 *                      through bit0),
 *               bit2 = advisory: the hold-out error came from the Gram
 *                      expansion of |Y_v - X_v W|^2 (pichol_holdout) and
 *                      cancellation there may cost it more than 1e-11 of
 *                      its relative accuracy (a well-fitted target: |R|^2
 *                      far below |Y_v|^2).  The calls that hold X and Y
 *                      (pichol_cv, pichol_exact_cv, pichol_cv_batch)
 *                      recompute such units from the residual itself
 *                      (pichol_holdout_direct) and clear the bit.
 *  - Results are bitwise reproducible from run to run (no floating-point
 *    atomics; every reduction has a fixed order).
 *  - All arithmetic is IEEE FP64, except where a call is asked for
 *    PICHOL_PREC_MIXED (below).
 *
 * Folds: k contiguous folds; fold f holds rows [start_f, start_{f+1}) with
 * sizes as numpy.array_split (the first n mod k folds get one extra row).
 * The training set of fold f is every other row.
 *
 * Tile-packed triangle ("packed" below)
 * -------------------------------------
 * A d x d lower triangle is stored as the lower triangle of 128 x 128 tiles:
 * nt = ceil(d/128) tile rows, tile (I,J) with J <= I at element offset
 * (I(I+1)/2 + J) * 16384, each tile column-major (entry (i,j) of the tile at
 * j*128 + i).  pichol_packed_elems(d) = nt(nt+1)/2 * 16384.  Rows and
 * columns at index >= d are padding: 1 on the diagonal, 0 elsewhere.  In a
 * factor, the strict upper part of every diagonal tile is 0; in a symmetric
 * input only entries with i >= j are read.
 * "dp" below is the padded order nt*128.
 *
 * Right-hand-side slab
 * --------------------
 * Solutions for q lambda values of one fold share a row-major dp x ldz
 * matrix, ldz = pichol_slab_cols(q, c) = q*c rounded up to a multiple of
 * 128; column t*c + j holds right-hand side j for lambda index t.
 */
#ifndef PICHOL_H
#define PICHOL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PICHOL_OK = 0,
  PICHOL_ERR_ARG = -1,       /* invalid argument or shape                  */
  PICHOL_ERR_WORKSPACE = -2, /* workspace missing or smaller than required */
  PICHOL_ERR_HIP = -3,       /* a HIP runtime call failed                  */
  PICHOL_ERR_NOT_PD = -4,    /* returned by pichol_check only              */
  PICHOL_ERR_DATA = -5       /* returned by pichol_check only: flags set   */
} pichol_status;

typedef enum {
  PICHOL_METHOD_INTERP = 1, /* piCholesky: Algorithm 1 + evaluation         */
  PICHOL_METHOD_EXACT = 2,  /* one exact factorization per grid value       */
  PICHOL_METHOD_GRAD = 4,   /* workspace flag: room for the *_grad calls    */
  PICHOL_METHOD_PINRMSE = 8 /* hold-out errors interpolated directly        */
} pichol_method;

/* Arithmetic of the factorizations (Sec. 3.2; Algorithm 1 step 1).
 *   PICHOL_PREC_FP64   everything in FP64 (FP64 MFMA).
 *   PICHOL_PREC_MIXED  the trailing updates of the blocked factorization,
 *                      which hold all but O(d^2 * 128) of its d^3/3 flops,
 *                      take their products on FP32 MFMA: factor entries are
 *                      rounded to FP32 as they are read and each 256-term
 *                      product is accumulated in FP32, then subtracted from
 *                      the FP64 trailing matrix.  Diagonal blocks, panels,
 *                      the fit, the solves and the hold-out errors stay FP64.
 *                      The factors then satisfy L L^T = H + lam I + E with
 *                      |E_ij| of the order of 1e-7 * sum_p |L_ip L_jp|. */
typedef enum {
  PICHOL_PREC_FP64 = 0,
  PICHOL_PREC_MIXED = 1
} pichol_precision;

/* Problem description shared by the pipeline calls.
 *   n, d, c   rows of X, features, right-hand sides (label columns);
 *             n >= k, d >= 1, 1 <= c
 *   k         folds, 2 <= k <= n
 *   g, r, q   sample lambdas, polynomial degree (0 <= r < g <= 32,
 *             r <= 7), dense grid size (q >= 1)
 *   normalize 1: H_f = X_tr^T X_tr / n_tr and B_f = X_tr^T Y_tr / n_tr;
 *             0: no division (the paper's X^T X, X^T y)
 *   precision a pichol_precision value for the factorizations
 *   basis     variable of the fitted polynomials in the pipeline calls:
 *             0 = tau = lambda / lam_ref (the polynomial space of Algorithm
 *             1: polynomials in lambda); 1 = log(lambda / lam_ref)
 *             (polynomials in log lambda, an alternative to the paper's
 *             basis for grids spanning many decades; every lambda must be
 *             positive).  The step calls pichol_fit, pichol_eval,
 *             pichol_solve_interp, pichol_fit_vec and pichol_eval_vec use
 *             basis 0.
 *   refine    0 .. PICHOL_MAX_REFINE steps of iterative refinement after
 *             the solves of the pipeline calls (pichol_cv_interp,
 *             pichol_cv_exact): R_t = B_f - (H_f + lambda_t I) W_t in FP64
 *             (H_f from the fold Gram blocks), then W_t += the solution of
 *             L L^T D = R_t with the same factor L (interpolated or
 *             exact).  With exact factors this recovers FP64 accuracy
 *             after a mixed-precision factorization.  With interpolated
 *             factors it moves W_t toward the exact ridge solution at
 *             lambda_t, i.e. toward exact cross-validation, converging
 *             where the interpolated factor is a close enough
 *             preconditioner (spectral radius of
 *             I - (Lhat Lhat^T)^{-1}(H_f + lambda_t I) below one).  Each
 *             step costs one residual product (2 d^2 q c flops per fold)
 *             and one pair of triangular solves.
 *   ldx, ldy  row-major leading dimensions of X (n x d) and Y (n x c),
 *             ldx >= d, ldy >= c                                            */
typedef struct {
  int64_t n, d, c;
  int32_t k, g, r, q;
  int32_t normalize;
  int32_t precision;
  int32_t refine;
  int32_t basis;
  int64_t ldx, ldy;
} pichol_problem;

#define PICHOL_MAX_REFINE 16

/* ---------------------------------------------------------------- layout */

/* Elements of one tile-packed triangle of order d (0 when d < 1). */
int64_t pichol_packed_elems(int64_t d);
/* Padded order nt*128 of a tile-packed triangle of order d. */
int64_t pichol_padded_order(int64_t d);
/* Column count of a right-hand-side slab holding q*c columns. */
int64_t pichol_slab_cols(int64_t q, int64_t c);

/* Dense -> packed (the vectorisation of a factor, Sec. 5: the tile-packed
 * triangle is this library's layout of a row of T in Algorithm 1).
 * A: nmat row-major d x d matrices (device, leading
 * dimension lda >= d, consecutive matrices lda*d apart); only entries with
 * i >= j are read.  P: nmat packed triangles (device), padding written as
 * above; the strict upper part of diagonal tiles is written as 0. */
pichol_status pichol_pack(int64_t d, int32_t nmat, const double *A,
                          int64_t lda, double *P, hipStream_t stream);

/* Packed -> dense lower triangle (inverse of the Sec. 5 vectorisation
 * above; for tests).  A receives nmat row-major d x d
 * matrices (device, leading dimension lda >= d) with zeros above the
 * diagonal. */
pichol_status pichol_unpack(int64_t d, int32_t nmat, const double *P,
                            double *A, int64_t lda, hipStream_t stream);

/* -------------------------------------------------------------- step calls */

/* Fold Gram matrices (Sec. 3.1: H = X^T X, g = X^T y).
 * In:  X n x d, Y n x c (device, row-major, leading dims in p).
 * Out (device):
 *   G   k x dp x dp: G[b] = X_b^T X_b over the rows of fold b, both
 *       triangles, stored as nt x nt column-major 128 x 128 tiles (tile
 *       (I,J) at (I*nt + J)*16384), padding 0;
 *   C   k x dp x c row-major: C[b] = X_b^T Y_b, padding rows 0;
 *   yy  k: yy[b] = sum of Y_b^2;
 *   H   k packed: H_f = sum_{b != f} G[b] (/ n_tr when normalize);
 *   B   k x dp x c row-major: B_f = sum_{b != f} C[b] (/ n_tr).
 * Sums over blocks run in increasing block order.  H must not overlap X, Y
 * or G: the call also keeps partial Gram tiles in it before writing H. */
pichol_status pichol_gram(const pichol_problem *p, const double *X,
                          const double *Y, double *G, double *C, double *yy,
                          double *H, double *B, hipStream_t stream);

/* Scratch bytes needed by pichol_potrf_shifted_batched for nmat*nshift
 * factorizations. */
size_t pichol_potrf_workspace(int32_t nmat, int32_t nshift);

/* Batched exact Cholesky of shifted matrices (Sec. 3.2; Algorithm 1 step 1).
 * In:  H nmat packed symmetric matrices of order d (device);
 *      lam nshift shifts (host).
 * Out: L nmat*nshift packed factors (device), factor (m,s) at
 *      (m*nshift + s) * pichol_packed_elems(d): L L^T = H_m + lam_s I on the
 *      first d rows/columns, lower triangular with positive diagonal;
 *      info nmat*nshift (device, int32), see the conventions above.
 * Blocked right-looking algorithm on 128-wide panels; the trailing updates
 * run on FP64 MFMA, or on FP32 MFMA when precision is PICHOL_PREC_MIXED.
 * ws: pichol_potrf_workspace(nmat, nshift) bytes. */
pichol_status pichol_potrf_shifted_batched(int64_t d, int32_t nmat,
                                           const double *H, int32_t nshift,
                                           const double *lam, double *L,
                                           int32_t *info, void *ws,
                                           size_t ws_bytes, int32_t precision,
                                           hipStream_t stream);

/* Least-squares polynomial fit of every factor entry (Algorithm 1 steps
 * 2-6).  The basis is the monomials 1, tau, ..., tau^r of
 * tau = lambda / lam_ref (the same polynomial space as monomials in lambda;
 * lam_ref > 0, normally the largest sample).  Theta = V^+ T with
 * V[s][j] = tau_s^j, the pseudo-inverse V^+ computed on the host in FP64 by
 * Householder QR.
 * In:  L nmat*g packed factors (device), factor (m,s) at (m*g + s)*S;
 *      lam_s g distinct sample values (host).
 * Out: theta nmat*(r+1) packed coefficient planes (device), plane (m,j) at
 *      (m*(r+1) + j)*S;
 *      theta_t (optional, may be NULL) the same planes with every tile
 *      stored row-major instead of column-major (used by the backward
 *      solve of pichol_solve_interp). */
pichol_status pichol_fit(int64_t d, int32_t nmat, int32_t g, int32_t r,
                         const double *lam_s, double lam_ref, const double *L,
                         double *theta, double *theta_t, hipStream_t stream);

/* Scratch bytes for pichol_eval with nlam values. */
size_t pichol_lambda_workspace(int32_t nlam);

/* Evaluate the fitted factor at nlam values (Sec. 3.3):
 * Lhat(m,t) = sum_j (lam_t/lam_ref)^j theta(m,j).
 * Out: Lhat nmat*nlam packed (device), (m,t) at (m*nlam + t)*S.
 * ws: pichol_lambda_workspace(nlam) bytes. */
pichol_status pichol_eval(int64_t d, int32_t nmat, int32_t r,
                          const double *theta, int32_t nlam,
                          const double *lam, double lam_ref, double *Lhat,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/* Scratch bytes for pichol_solve_interp: the q scaled lambdas, the inverses
 * of every diagonal 128 x 128 block of every interpolated factor
 * (nmat * q * ceil(d/128) * 131072 bytes), and a second slab of the same
 * shape as Z (the forward solves leave their blocks there).
 * Returns 0 when an argument is below 1. */
size_t pichol_solve_interp_workspace(int64_t d, int32_t nmat, int32_t q,
                                     int32_t c);

/* Interpolated solves for all q grid values of nmat folds (Sec. 3.2 applied
 * to the evaluated factor of Sec. 3.3), without materialising the factors:
 * forward substitution Lhat_t U = B then back substitution Lhat_t^T W = U,
 * blocked over 128-row tiles.  The diagonal blocks of every Lhat_t are
 * evaluated and inverted once; each step multiplies by the stored inverses,
 * and the off-diagonal updates of all q values are one FP64 MFMA product
 * with the r+1 coefficient planes.
 * In:  theta, theta_t from pichol_fit (device); B nmat x dp x c row-major
 *      (device, padding rows 0); lam q values (host).
 * Out: Z nmat slabs of dp x pichol_slab_cols(q,c) (device): W for every
 *      (fold, lambda); flags nmat*q (device, int32), zeroed then set.
 * ws: pichol_solve_interp_workspace(d, nmat, q, c) bytes. */
pichol_status pichol_solve_interp(int64_t d, int32_t nmat, int32_t c,
                                  int32_t r, const double *theta,
                                  const double *theta_t, const double *B,
                                  int32_t q, const double *lam,
                                  double lam_ref, double *Z, int32_t *flags,
                                  void *ws, size_t ws_bytes,
                                  hipStream_t stream);

/* Exact solves with given factors (Sec. 3.2): for fold m and index t,
 * L(m,t) W = B_m by forward then back substitution.
 * In:  L nmat*nper packed factors (device), (m,t) at (m*nper + t)*S;
 *      B nmat x dp x c row-major (device).
 * Out: Z nmat slabs dp x pichol_slab_cols(nper,c) (device);
 *      flags nmat*nper (device), zeroed then set. */
pichol_status pichol_solve_factors(int64_t d, int32_t nmat, int32_t nper,
                                   int32_t c, const double *L,
                                   const double *B, double *Z,
                                   int32_t *flags, hipStream_t stream);

/* Scratch bytes for pichol_holdout. */
size_t pichol_holdout_workspace(int64_t d, int32_t nmat, int32_t q,
                                int32_t c);

/* Hold-out error of every (fold, lambda), the quantity whose mean over the
 * folds k-fold cross-validation minimises over lambda (Sec. 3.1; its mean
 * squared form, the hold-out errors of Sec. 6.5): with R = Y_v - X_v W,
 * sse = |R|_F^2 computed as |Y_v|^2 - 2<W, X_v^T Y_v> + <W, X_v^T X_v W>,
 * err = sse / (nv * c).  The expansion reads the validation Gram matrices
 * of the Gram step instead of X_v; where its terms cancel (estimated
 * rounding 4 eps |Y_v|^2 (sqrt(nv) + sqrt(dp)) above 1e-11 sse, or
 * sse <= 0) flags bit2 is set (see pichol_holdout_direct).
 * In:  Z nmat slabs (device, as produced by the solve calls);
 *      G, C, yy of the validation blocks (device, as from pichol_gram;
 *      G is symmetric and only its tiles (I,J) with J <= I are read);
 *      nv nmat validation row counts (host).
 * Out: err nmat*q (device, FP64); flags nmat*q (device): bit0 is OR-ed in
 *      when err is not finite.
 * ws: pichol_holdout_workspace(d, nmat, q, c) bytes. */
pichol_status pichol_holdout(int64_t d, int32_t nmat, int32_t c, int32_t q,
                             const double *Z, const double *G,
                             const double *C, const double *yy,
                             const int64_t *nv, double *err, int32_t *flags,
                             void *ws, size_t ws_bytes, hipStream_t stream);

/* pichol_holdout for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, results and kernels, with no workspace argument.  The
 * partial sums live in a static device array of the library of
 * PICHOL_HOLDOUT_SCRATCH_BYTES (16 MiB), one per GPU, held until the process
 * ends; the call allocates nothing.  Calls whose partial sums need more
 * (pichol_holdout_workspace(d, nmat, q, c) above the limit; at d = 4096,
 * q = 64, c = 10 that is nmat > 12) return PICHOL_ERR_WORKSPACE before
 * anything is enqueued, with a message in pichol_last_error.  Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different threads) race and give wrong
 * results; calls in stream order are safe.  The array keeps the last call's
 * partial sums; each call writes every entry it later reads. */
#define PICHOL_HOLDOUT_SCRATCH_BYTES (16u << 20)
pichol_status pichol_holdout_noalloc(int64_t d, int32_t nmat, int32_t c,
                                     int32_t q, const double *Z,
                                     const double *G, const double *C,
                                     const double *yy, const int64_t *nv,
                                     double *err, int32_t *flags,
                                     hipStream_t stream);

/* Scratch bytes for pichol_holdout_direct (0 on invalid arguments). */
size_t pichol_holdout_direct_workspace(const pichol_problem *p);

/* Hold-out error of every (fold, lambda) from its definition (Sec. 3.1):
 * R = Y_v - X_v W, err = |R|_F^2 / (nv * c), the product X_v W on FP64
 * MFMA (2 nv d q c flops per fold; the squares summed per 128-row block,
 * then over the blocks in order).  This is the form the oracle takes; the
 * pipeline calls with X at hand use it for the units flagged bit2 by the
 * Gram expansion.
 * In:  p (n, d, c, k, q, normalize, ldx, ldy are used), X, Y (device, as
 *      for pichol_gram); Z k slabs of dp x pichol_slab_cols(q, c) (device,
 *      as produced by the solve calls, rows >= d zero).
 * Out: err k*q (device); flags k*q (device, read and updated): bit2
 *      cleared, bit0 OR-ed in when err is not finite.
 * ws: pichol_holdout_direct_workspace(p) bytes. */
pichol_status pichol_holdout_direct(const pichol_problem *p, const double *X,
                                    const double *Y, const double *Z,
                                    double *err, int32_t *flags, void *ws,
                                    size_t ws_bytes, hipStream_t stream);

/* Copy slabs to the k x q x d x c weight layout of the ridge solutions
 * theta(lambda) of Sec. 3.1: W[m][t][i][j] = Z[m][i][t*c + j]. */
pichol_status pichol_slab_to_weights(int64_t d, int32_t nmat, int32_t q,
                                     int32_t c, const double *Z, double *W,
                                     hipStream_t stream);

/* --------------------------------------------------------------- pipelines */

/* Workspace bytes for the pipeline calls below with the given method(s)
 * (a bitwise OR of pichol_method values: one workspace sized for both
 * serves both). */
pichol_status pichol_workspace_size(const pichol_problem *p, int32_t methods,
                                    size_t *bytes);

/* Stage 1: the fold Gram matrices H_f = X_tr^T X_tr, B_f = X_tr^T Y_tr of
 * Sec. 3.1 (and the validation blocks' G, C, |Y_v|^2) into the workspace,
 * as pichol_gram computes them. */
pichol_status pichol_cv_gram(const pichol_problem *p, const double *X,
                             const double *Y, void *ws, size_t ws_bytes,
                             hipStream_t stream);

/* Stage 2 (piCholesky, Algorithm 1 and the evaluation of Sec. 3.3): from
 * the Grams in ws, the g sample factorizations per fold (Algorithm 1 step
 * 1), the least-squares fit of every factor entry (steps 2-6; the
 * tile-packed factor is the row of T), the evaluation at the q grid values
 * fused into the forward and back substitutions of Sec. 3.2, and the
 * hold-out errors of Sec. 3.1 (Gram expansion, see pichol_holdout).
 *   lam_s (host, g distinct values), lam_grid (host, q), lam_ref > 0
 *   err  k*q (device) hold-out mean squared error
 *   W    k*q*d*c (device) weights, or NULL
 *   info k*g (device) status of the sample factorizations
 *   flags k*q (device)
 * When d spans more than 8 tiles of 128, the fit and the diagonal-block
 * inverses of the finished columns run on a second stream that the library
 * creates once per device (default priority); it is forked from and joined
 * back into `stream` by events inside the call, so the call stays ordered
 * on `stream` and may be captured into a graph.  Calls from several host
 * threads take a library mutex for their host part and are serialised
 * there. */
pichol_status pichol_cv_interp(const pichol_problem *p, const double *lam_s,
                               const double *lam_grid, double lam_ref,
                               void *ws, size_t ws_bytes, double *err,
                               double *W, int32_t *info, int32_t *flags,
                               hipStream_t stream);

/* Stage 2 (exact baseline, the "Chol" method of the comparison in
 * Sec. 6.2): one exact Cholesky factorization per (fold, grid value) of
 * H_f + lambda_t I (Sec. 3.2), the forward and back substitutions, and the
 * hold-out errors of Sec. 3.1 (Gram expansion, see pichol_holdout).
 * info is k*q. */
pichol_status pichol_cv_exact(const pichol_problem *p, const double *lam_grid,
                              void *ws, size_t ws_bytes, double *err,
                              double *W, int32_t *info, int32_t *flags,
                              hipStream_t stream);

/* Differentiation form: pichol_cv_interp, then the derivative of every
 * hold-out error with respect to log lambda through the interpolated factor
 * (the polynomial of Sec. 3.3 is differentiable in lambda):
 *   A = Lhat Lhat^T, theta = A^{-1} B_f, R = Y_v - X_v theta,
 *   z = A^{-1} X_v^T R (X_v^T R = C_v - G_v theta from the validation
 *   block's Gram matrices; one more pair of interpolated solves),
 *   d err / d lambda = 2/(n_v c) (<dLhat^T z, Lhat^T theta>
 *                                + <Lhat^T z, dLhat^T theta>),
 *   dLhat = sum_j j tau^(j-1) / lam_ref Theta_j,
 *   dlog = lambda * d err / d lambda.
 * lam_ref and the samples stay fixed (they define the fit).  All FP64.
 * Out: dlog k*q (device) besides the outputs of pichol_cv_interp.
 * p->refine must be 0.  ws: pichol_workspace_size with
 * PICHOL_METHOD_INTERP | PICHOL_METHOD_GRAD. */
pichol_status pichol_cv_interp_grad(const pichol_problem *p,
                                    const double *lam_s,
                                    const double *lam_grid, double lam_ref,
                                    void *ws, size_t ws_bytes, double *err,
                                    double *dlog, double *W, int32_t *info,
                                    int32_t *flags, hipStream_t stream);

/* The same derivative for the exact method of Sec. 3.2 (dA/dlambda = I):
 * d err / d lambda = 2/(n_v c) <z, theta>, z = (H_f + lambda I)^{-1} X_v^T R,
 * i.e. the exact gradient the interpolated one approximates.
 * ws: pichol_workspace_size with PICHOL_METHOD_EXACT | PICHOL_METHOD_GRAD. */
pichol_status pichol_cv_exact_grad(const pichol_problem *p,
                                   const double *lam_grid, void *ws,
                                   size_t ws_bytes, double *err, double *dlog,
                                   double *W, int32_t *info, int32_t *flags,
                                   hipStream_t stream);

/* The hold-out-error variant of Algorithm 1 (PINRMSE, Sec. 6.5 and its
 * supplement): the exact hold-out errors at the g samples (exact Cholesky,
 * as pichol_cv_exact at lambda = lam_s) take the place of the g x D matrix
 * T, i.e. the polynomial of degree r in tau = lambda/lam_ref is fitted to
 * the g errors of each fold and evaluated at the q grid values.
 * Needs the Gram matrices in ws (pichol_cv_gram).
 * Out: err k*q (device) the interpolated hold-out errors; err_s k*g
 *      (device, may be NULL) the exact errors at the samples; info, flags
 *      k*g (device) the status of the sample factorizations and solves.
 * ws: pichol_workspace_size with PICHOL_METHOD_PINRMSE. */
pichol_status pichol_cv_pinrmse(const pichol_problem *p, const double *lam_s,
                                const double *lam_grid, double lam_ref,
                                void *ws, size_t ws_bytes, double *err,
                                double *err_s, int32_t *info, int32_t *flags,
                                hipStream_t stream);

/* piCholesky k-fold cross-validation of ridge regression from X and Y
 * (Sec. 3.1 problem, Sec. 3.3 method): pichol_cv_gram followed by
 * pichol_cv_interp, then the units flagged bit2 recomputed from the
 * residual Y_v - X_v W (pichol_holdout_direct), so that every hold-out
 * error is accurate to the FP64 level whatever the fit's quality.  X and Y
 * are read again by that last step. */
pichol_status pichol_cv(const pichol_problem *p, const double *X,
                        const double *Y, const double *lam_s,
                        const double *lam_grid, double lam_ref, void *ws,
                        size_t ws_bytes, double *err, double *W,
                        int32_t *info, int32_t *flags, hipStream_t stream);

/* Exact k-fold cross-validation of ridge regression from X and Y
 * (Sec. 3.1 problem, Sec. 3.2 solves; the "Chol" baseline of Sec. 6.2):
 * pichol_cv_gram followed by pichol_cv_exact, then the units flagged bit2
 * recomputed from the residual as in pichol_cv. */
pichol_status pichol_exact_cv(const pichol_problem *p, const double *X,
                              const double *Y, const double *lam_grid,
                              void *ws, size_t ws_bytes, double *err,
                              double *W, int32_t *info, int32_t *flags,
                              hipStream_t stream);

/* ------------------------------------------------- vectorisation layouts */

/* Layouts of Sec. 5 for the vector that holds one factor as a row of T
 * (the layout comparison of Table 1):
 *   ROWWISE    entry (i,j), j <= i, at i(i+1)/2 + j
 *   FULL       the d x d matrix, row-major, zeros above the diagonal
 *   RECURSIVE  eq. (recursive): split at half = d/2 into the square block
 *              L12 = rows [half,d) x columns [0,half) stored first,
 *              row-major, then L11, then L22, each split the same way until
 *              the order is at most h0, where rows are concatenated (d need
 *              not be a power of two: L12 is then (d-half) x half)
 *   TILE       the tile-packed triangle the factorization writes (the
 *              library's own layout: no conversion needed)
 * Vector lengths are rounded up to a multiple of 4; entries past the
 * layout's own length are not written. */
typedef enum {
  PICHOL_LAYOUT_ROWWISE = 1,
  PICHOL_LAYOUT_FULL = 2,
  PICHOL_LAYOUT_RECURSIVE = 3,
  PICHOL_LAYOUT_TILE = 4
} pichol_layout;

/* Length of one vectorised factor of order d in the layout (0 if invalid). */
int64_t pichol_vector_length(int64_t d, int32_t layout);

/* Tile-packed factors (device, nmat of them) -> their vectors in `layout`
 * (Sec. 5 and Table 1: ROWWISE, FULL or RECURSIVE block vectorisation with
 * threshold h0 >= 1), T nmat x
 * pichol_vector_length(d, layout) (device). */
pichol_status pichol_vectorize(int64_t d, int32_t nmat, const double *L,
                               int32_t layout, int32_t h0, double *T,
                               hipStream_t stream);

/* The fit of pichol_fit (Algorithm 1 steps 2-6) on flat vectors of length
 * N (a multiple of 4), as in the layout comparison of Table 1:
 * theta(m, j) = sum_s P[j][s] T(m, s), T nmat*g x N, theta nmat*(r+1) x N
 * (device). */
pichol_status pichol_fit_vec(int64_t N, int32_t nmat, int32_t g, int32_t r,
                             const double *lam_s, double lam_ref,
                             const double *T, double *theta,
                             hipStream_t stream);

/* The evaluation of pichol_eval (Sec. 3.3) on flat vectors, as in the
 * layout comparison of Table 1: out(m, t) =
 * sum_j (lam_t/lam_ref)^j theta(m, j), out nmat*nlam x N (device).
 * ws: pichol_lambda_workspace(nlam) bytes. */
pichol_status pichol_eval_vec(int64_t N, int32_t nmat, int32_t r,
                              const double *theta, int32_t nlam,
                              const double *lam, double lam_ref, double *out,
                              void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- batching */

/* One independent ridge problem of a batch: the arguments of the
 * single-problem pipeline (pichol_cv_gram followed by pichol_cv_interp or
 * pichol_cv_exact) gathered in one record.  p.refine must be 0; p.precision
 * applies to the problem's factorizations.  X, Y, err, W, info, flags are
 * device pointers as in those calls; lam_s (g values, interpolated method
 * only) and lam_grid (q values) are host arrays read during the call. */
typedef struct {
  pichol_problem p;
  const double *X, *Y;
  const double *lam_s;
  const double *lam_grid;
  double lam_ref;
  double *err;     /* k*q                                              */
  double *W;       /* k*q*d*c, or NULL                                 */
  int32_t *info;   /* k*g (interpolated) or k*q (exact)                */
  int32_t *flags;  /* k*q                                              */
} pichol_batch_item;

/* Scheduling knobs of a batch (pass NULL for the defaults; the values an
 * autotuner picks per batch signature).
 *   streams      concurrent streams for independent buckets, 1..4 (0 = 4)
 *   order        0: buckets by decreasing estimated work (d^3 x
 *                factorizations), assigned to the least-loaded stream;
 *                1: input order, round-robin over the streams
 *   panel_group  per d bucket: panel_group[nt-1] (nt = ceil(d/128) <= 32)
 *                panels per delayed trailing update in that bucket's
 *                factorizations, 1..8, or 0 for PICHOL_OPT_PANEL_GROUP
 *   solve_form   per d bucket: the form of its interpolated solves, 1
 *                (stacked) or 2 (per lambda), or 0 for
 *                PICHOL_OPT_SOLVE_FORM */
typedef struct {
  int32_t streams;
  int32_t order;
  int32_t panel_group[32];
  int32_t solve_form[32];
} pichol_batch_tuning;

/* Many independent problems of uneven size in one call (Sec. 3.3's method
 * applied to a workload of many ridge problems).  Problems that share d, c,
 * k, g, r, q, precision and, for the interpolated method, the scaled sample
 * and grid values lambda/lam_ref to within 8 ulps (so the fit's
 * pseudo-inverse and the evaluation weights are shared; the bucket uses its
 * first problem's scaled values) form a bucket: every fold, lambda and
 * problem of a bucket runs in the same launches (the stacked matrices of
 * the bucket are one batch for the factorization, fit, solve and hold-out
 * kernels; each problem keeps its own shifts lambda_s, fold split and hold-out
 * counts).  Buckets are independent and run concurrently on library-owned
 * streams (default priority, created on first use per device), forked from
 * and joined back to `stream` with events, so the call is capturable into a
 * HIP graph (pichol_cv_batch_graph).  Results equal those of the
 * single-problem pipeline bit for bit when the scaled values agree exactly,
 * and to within the effect of those few ulps otherwise.
 *   method  PICHOL_METHOD_INTERP or PICHOL_METHOD_EXACT (one of them)
 *   ws      pichol_batch_workspace_size bytes: each bucket has its own
 *           region, laid out as the single-problem workspace of its stacked
 *           problems. */
pichol_status pichol_batch_workspace_size(int32_t nprob,
                                          const pichol_batch_item *items,
                                          int32_t method, size_t *bytes);
pichol_status pichol_cv_batch(int32_t nprob, const pichol_batch_item *items,
                              int32_t method, const pichol_batch_tuning *tune,
                              void *ws, size_t ws_bytes, hipStream_t stream);

/* Number of buckets the call above forms (host only, for inspection). */
int32_t pichol_batch_buckets(int32_t nprob, const pichol_batch_item *items,
                             int32_t method);

/* The whole batch as one HIP graph: pichol_cv_batch captured on a private
 * stream and instantiated.  The graph records the items' pointers and the
 * lambda values as they are at this call; each pichol_graph_launch replays
 * every launch of the batch with one host call.  Per-kernel profiling must
 * be off while a graph is built. */
typedef struct pichol_graph_s *pichol_graph;
pichol_status pichol_cv_batch_graph(int32_t nprob,
                                    const pichol_batch_item *items,
                                    int32_t method,
                                    const pichol_batch_tuning *tune, void *ws,
                                    size_t ws_bytes, pichol_graph *graph);
pichol_status pichol_graph_launch(pichol_graph graph, hipStream_t stream);
pichol_status pichol_graph_destroy(pichol_graph graph);

/* Capture any sequence of library calls made on `stream` (which must not be
 * the legacy null stream) between these two calls into one HIP graph, e.g.
 * the piCholesky stage of a repeated cross-validation: every launch of the
 * sequence then replays with one pichol_graph_launch.  Host arrays
 * (lambda values) are read during the capture and recorded in the graph.
 * The look-ahead side stream and per-kernel profiling must be off during a
 * capture; other threads' work is not captured (thread-local capture).
 * pichol_cv_interp (and pichol_cv) called on a capturing stream runs all of
 * its work on that stream: it does not fork the second stream it uses
 * above twelve tile columns (same results). */
pichol_status pichol_graph_begin(hipStream_t stream);
pichol_status pichol_graph_end(hipStream_t stream, pichol_graph *graph);

/* ------------------------------------------------------------------ misc */

/* Synchronise the stream and inspect info/flags (device arrays, either may
 * be NULL): PICHOL_ERR_NOT_PD when some info is non-zero, PICHOL_ERR_DATA
 * when some flag has bit0 or bit1 set (bit2 is advisory),
 * PICHOL_ERR_HIP on a runtime failure. */
pichol_status pichol_check(const int32_t *info, int64_t n_info,
                           const int32_t *flags, int64_t n_flags,
                           hipStream_t stream);

/* Static description of a status code. */
const char *pichol_status_string(pichol_status s);

/* Text of the last HIP error the library saw on this thread, or of the
 * last argument error that carries a message ("" if none). */
const char *pichol_last_error(void);

/* ---------------------------------------------------------------- options */

typedef enum {
  /* 0 (default) or 1.  When 1, the blocked factorizations run the bulk of
   * each trailing update on a library-owned side stream (default priority,
   * created with a few events on first use on each device), joined back to
   * the caller's stream by events, so the next panels' diagonal
   * factorizations overlap it.  Results are identical either way. */
  PICHOL_OPT_LOOKAHEAD = 1,
  /* 1..8 (default 4): the blocked factorizations take their 128-wide
   * panels in groups of this many.  Inside a group, each panel's column
   * first receives the group's earlier panels (a rank-128u update of that
   * column); after the group, one rank-(128 x group) update reaches the
   * rest of the trailing matrix, so larger groups read and write the
   * trailing matrix fewer times.  With the look-ahead option, the update
   * of the next group's columns stays on the caller's stream and the rest
   * of each group's trailing update runs on the side stream.  Results differ
   * only by the rounding order of the trailing sums. */
  PICHOL_OPT_PANEL_GROUP = 2,
  /* 0 (default), 1 or 2: the form of the interpolated solves (Sec. 3.2
   * with the factors of Sec. 3.3).  2: per lambda, each step evaluating
   * every lambda's coefficient tile in registers and multiplying it with
   * that lambda's columns only (padded to 16 per lambda), with the next
   * diagonal block solved inside the same launch; 1: stacked, each step one
   * product of the r+1 coefficient tiles with every column scaled by the
   * powers of tau (q*c columns rounded up to 128), and a launch of its own
   * for each diagonal block; 0: per call, by their product counts (per
   * lambda when (r+1) * slab columns >= 24 q ceil(c/16), e.g. c = 10;
   * stacked for c = 1).  Results differ only by rounding. */
  PICHOL_OPT_SOLVE_FORM = 3
} pichol_option;

/* Set a process-wide option; PICHOL_ERR_ARG for an unknown option or
 * value. */
pichol_status pichol_set_option(int32_t option, int32_t value);

/* Current value of an option, or -1 for an unknown option. */
int32_t pichol_get_option(int32_t option);

/* ---------------------------------------------------- accuracy diagnostics */

/* Scratch bytes for pichol_factor_nrmse. */
size_t pichol_factor_nrmse_workspace(int64_t d, int32_t nmat);

/* Accuracy of fitted factors (the NRMSE section of Sec. 6): for each of
 * nmat pairs of packed factors of order d,
 *   out[m] = sqrt(sum (Lhat_m - L_m)^2) / sqrt(sum (L_m - mean L_m)^2)
 * over the d(d+1)/2 entries with i >= j (padding excluded), mean over the
 * same entries; predicting every entry by the mean gives 1.
 * In:  Lhat, L nmat packed factors each (device), e.g. pichol_eval at some
 *      lambdas and pichol_potrf_shifted_batched at the same lambdas.
 * Out: out nmat doubles (device); inf/NaN when L is constant.
 * ws: pichol_factor_nrmse_workspace(d, nmat) bytes.  Per-tile statistics
 * are merged in a fixed order, so results are reproducible. */
pichol_status pichol_factor_nrmse(int64_t d, int32_t nmat, const double *Lhat,
                                  const double *L, double *out, void *ws,
                                  size_t ws_bytes, hipStream_t stream);

/* Hold-out NRMSE (the normalised error of the Sec. 6.5 hold-out tables)
 * from the hold-out MSE of a cross-validation call:
 *   nrmse[f*q + t] = sqrt(err[f*q + t] * n_v c / SST_f),
 * SST_f the sum over fold f's rows and the c columns of (Y - the fold's
 * column mean)^2, so predicting every label by that mean gives 1.
 * In:  p (n, c, k, q, ldy are used), Y n x c (device, row-major, ldy);
 *      err k x q (device).  Out: nrmse k x q (device). */
pichol_status pichol_holdout_nrmse(const pichol_problem *p, const double *Y,
                                   const double *err, double *nrmse,
                                   hipStream_t stream);

/* ------------------------------------------------------------- profiling */

/* Per-kernel timing with HIP events, for benchmarks and tuning.  While
 * enabled, every kernel launch the library makes is bracketed by two HIP
 * events recorded on the launch stream; the first `capacity` launches are
 * recorded, later ones are not.  pichol_profile_start creates the 2*capacity
 * events (it allocates; the compute calls never do) and clears earlier
 * records.  Recording is process-wide: enable it only while one host thread
 * issues library calls. */
pichol_status pichol_profile_start(int32_t capacity);

/* Stop recording; the records stay readable. */
pichol_status pichol_profile_stop(void);

/* Wait for the recorded events and aggregate them by kernel name.  Fills
 * up to `max` entries of names / launches / total_ms (any may be NULL;
 * names stay valid until the next profiling call) and returns the number
 * of distinct kernels, or -1 on a HIP error. */
int32_t pichol_profile_summary(int32_t max, const char **names,
                               int64_t *launches, double *total_ms);

/* Destroy the events and records. */
pichol_status pichol_profile_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* PICHOL_H */
