// Host-side launchers of the gfx950 kernels.  Each launcher enqueues its
// kernels on `stream` and returns the HIP launch status; shapes are
// validated by the C-ABI layer before any launcher runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pichol {

// Opt-in per-kernel timing (pichol_profile_* in the C-ABI): while enabled,
// every launch made through PICHOL_LAUNCH is bracketed by a pair of HIP
// events recorded on the launch stream.  Disabled, it costs one flag test.
struct ProfScope {
  const char* name;
  hipStream_t stream;
  int slot;
  ProfScope(const char* n, hipStream_t s);
  ~ProfScope();
};

#define PICHOL_LAUNCH(K, GRID, BLOCK, SHMEM, STREAM, ...)                 \
  do {                                                                    \
    ::pichol::ProfScope prof_scope_(#K, STREAM);                          \
    hipLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);       \
  } while (0)

hipError_t record_hip_error_code(hipError_t e);

// Library options (pichol_set_option).
int option_lookahead();
int option_panel_group();
int option_solve_form();
inline int record_hip_error(hipError_t e) {
  (void)record_hip_error_code(e);
  return -3;  // PICHOL_ERR_HIP
}

// ---- layout (k_layout.hip)
hipError_t launch_store_doubles(const double* host, int n, double* dev,
                                hipStream_t s);
hipError_t launch_pack(int64_t d, int nmat, const double* A, int64_t lda,
                       double* P, hipStream_t s);
hipError_t launch_unpack(int64_t d, int nmat, const double* P, double* A,
                         int64_t lda, hipStream_t s);
hipError_t launch_slab_to_weights(int64_t d, int nmat, int q, int c,
                                  int64_t ldz, const double* Z, double* W,
                                  hipStream_t s);
hipError_t launch_copy_i32(int64_t n, const int* src, int* dst, hipStream_t s);
// layout: 1 row-wise, 2 full matrix, 3 recursive (threshold h0); N is the
// vector length of one factor in that layout.
hipError_t launch_vectorize(int64_t d, int nmat, const double* P, int layout,
                            int64_t h0, int64_t N, double* T, hipStream_t s);

// ---- Gram (k_gram.hip)
struct FoldSplit {
  int k;
  int64_t start[65];  // start[f] .. start[f+1] rows of fold f (k <= 64)
  double scale[64];   // 1/n_tr or 1
};
// Looks up, once per device, the device facts the Gram launch depends on
// (for callers about to start a stream capture).
void prepare_gram();
hipError_t launch_gram(const double* X, int64_t ldx, const double* Y,
                       int64_t ldy, int64_t d, int64_t c,
                       const FoldSplit& fs, double* G, double* C, double* yy,
                       double* H, double* B, hipStream_t s);

// ---- POTRF (k_potrf.hip)
// Where the factorizations take their matrices: factor f is
// H(f / nshift) + lam[((f / nshift) / lam_group) * nshift + f % nshift] I,
// H tile-packed with identity padding.  The first launch that touches a
// tile reads it from H (adding the shift on the diagonal) and writes L, so
// no shifted copy of H is ever made.
struct ShiftSrc {
  const double* H;
  int nshift;
  const double* lam;  // device
  int lam_group;
};
// lookahead: 1 runs the bulk of each trailing update on the library's side
// stream (see k_potrf.hip), 0 keeps everything on s.  group: panels per
// delayed trailing update (0: the library option).  info is written for
// every factor (0, or the 1-based index of the first non-positive pivot).
// linv_ws: nfac * 16384 doubles of scratch, or with keep_linv
// nfac * ceil(d/128) * 16384 doubles that keep the inverse of every
// diagonal tile, (f * nt + I) * 16384 for tile I of factor f.
// Called by launch_potrf_blocked once the launches that finish column `col`
// (its diagonal tile and panel) are enqueued on the stream: every tile of
// columns 0 .. col is then final once the stream reaches that point.
struct PanelHook {
  int col;
  hipError_t (*fn)(void* ctx);
  void* ctx;
};
hipError_t launch_potrf_blocked(int64_t d, int nfac, const ShiftSrc& src,
                                double* L, int* info, double* linv_ws,
                                int keep_linv, int mixed, int lookahead,
                                int group, hipStream_t s,
                                const PanelHook* hook = nullptr);

// ---- fit / evaluate (k_fit.hip)
struct FitCoef {
  int g, m;          // samples, planes (r+1)
  double P[8][32];   // pseudo-inverse of V: m x g
};
hipError_t launch_fit(int64_t d, int nmat, const FitCoef& fc, const double* L,
                      double* theta, double* theta_t, hipStream_t s);
// The fit of the tiles of columns J0 .. J1-1 only.
hipError_t launch_fit_cols(int64_t d, int nmat, const FitCoef& fc,
                           const double* L, double* theta, double* theta_t,
                           int J0, int J1, hipStream_t s);
hipError_t launch_fit_flat(int64_t N, int nmat, const FitCoef& fc,
                           const double* T, double* theta, hipStream_t s);
hipError_t launch_eval_flat(int64_t N, int nmat, int m, const double* theta,
                            int nlam, const double* tau_dev, double* out,
                            hipStream_t s);
hipError_t launch_pinrmse(int nmat, const FitCoef& fc, int q,
                          const double* tau_dev, const double* es, double* err,
                          hipStream_t s);
hipError_t launch_eval(int64_t d, int nmat, int m, const double* theta,
                       int nlam, const double* tau_dev, double* Lhat,
                       hipStream_t s);

// ---- triangular solves (k_trsm.hip)
hipError_t launch_slab_init(int64_t d, int nmat, int q, int c, int64_t ldz,
                            const double* B, double* Z, int* flags,
                            hipStream_t s);
// The inverted diagonal blocks of tile rows i0 .. i1-1 of every
// interpolated factor, as pichol_solve_interp prepares them.
hipError_t launch_diag_inv(int64_t d, int nmat, int M, const double* theta,
                           int q, const double* tau_dev, double* dinv,
                           int* flags, int i0, int i1, hipStream_t s);
// The form of the interpolated solves for M planes, q values, c columns
// and slab width ldz: requested 1 (stacked) or 2 (per lambda) as given,
// 0 the PICHOL_OPT_SOLVE_FORM option, whose 0 is the automatic choice.
int solve_form_for(int M, int q, int c, int64_t ldz, int requested);
// The interpolated solves of every fold at the q values (Z: right-hand
// sides in, solutions out; X: second slab) in the form solve_form_for
// gives.  With the per-lambda form, fwd_from > 0 skips the forward steps
// launch_solve_fwd has already run.
hipError_t launch_solve_interp(int64_t d, int nmat, int c, int m,
                               const double* theta, const double* theta_t,
                               int q, const double* tau_dev, int64_t ldz,
                               double* Z, double* X, int* flags, double* dinv,
                               int prepare, hipStream_t s, int fwd_from = 0,
                               int form = 0);
// Forward steps i0 .. i1-1 of the per-lambda form (i0 = 0 also solves the
// first diagonal block).  narrow: two units per workgroup in every launch,
// for steps that do not share the GPU with a factorization.
hipError_t launch_solve_fwd(int64_t d, int nmat, int c, int M,
                            const double* theta, int q, const double* tau_dev,
                            int64_t ldz, double* Z, double* X,
                            const double* dinv, int i0, int i1, hipStream_t s,
                            bool narrow = false);
// With linv (the kept inverses of the factors' diagonal tiles, see
// launch_potrf_blocked) and a second slab X, each diagonal step is a product
// with a stored inverse; without them it is a substitution in place.
hipError_t launch_solve_factors(int64_t d, int nmat, int nper, int c,
                                const double* L, int64_t ldz, double* Z,
                                int* flags, const double* linv, double* X,
                                hipStream_t s);

// ---- hold-out (k_holdout.hip)
struct HoldoutNorm {
  int nmat;
  double count[64];  // n_v * c per fold
};
// The hold-out products split their 128-row-block sums over this many
// ranges of column blocks (more, shorter workgroups); partial sums hold
// nmat * nt * HOLDOUT_KSPLIT * ldz doubles.
constexpr int HOLDOUT_KSPLIT = 8;
hipError_t launch_holdout_partial(int64_t d, int nmat, int c, int q,
                                  int64_t ldz, const double* Z,
                                  const double* G, const double* C,
                                  double* partial, hipStream_t s);
hipError_t launch_holdout_final(int64_t d, int nmat, int c, int q, int64_t ldz,
                                const double* partial, const double* yy,
                                const HoldoutNorm& hn, double* err, int* flags,
                                hipStream_t s);
hipError_t launch_holdout(int64_t d, int nmat, int c, int q, int64_t ldz,
                          const double* Z, const double* G, const double* C,
                          const double* yy, const HoldoutNorm& hn,
                          double* partial, double* err, int* flags,
                          hipStream_t s);
// Flag bit 2: the Gram-form hold-out error of the unit lost accuracy to
// cancellation (its estimated rounding exceeds 1e-11 of the result).
constexpr int FLAG_CANCEL = 4;
// Row blocks of 128 of the largest fold: the direct hold-out partial sums
// hold nmat * holdout_direct_rowblocks(fs) * ldz doubles.
int64_t holdout_direct_rowblocks(const FoldSplit& fs);
// Hold-out errors from the residual R = Y_v - X_v W itself (fold m's
// validation rows fs.start[m] .. fs.start[m+1]-1 of X and Y, its solutions
// in slab m of Z): every unit, or (only_flagged) those marked FLAG_CANCEL.
// The recomputed units' FLAG_CANCEL bit is cleared.
hipError_t launch_holdout_direct(int64_t d, int nmat, int c, int q,
                                 int64_t ldz, const double* Z, const double* X,
                                 int64_t ldx, const double* Y, int64_t ldy,
                                 const FoldSplit& fs, const HoldoutNorm& hn,
                                 double* partial, double* err, int* flags,
                                 int only_flagged, hipStream_t s);

// ---- iterative refinement (k_refine.hip)
hipError_t launch_full_h(int64_t d, const FoldSplit& fs, const double* G,
                         double* Hf, hipStream_t s);
hipError_t launch_residual(int64_t d, int nmat, int q, int c, int64_t ldz,
                           const double* Hf, const double* B,
                           const double* lam_dev, const double* Z, double* R,
                           hipStream_t s);
hipError_t launch_slab_add(int64_t d, int nmat, int64_t ldz, const double* D,
                           double* Z, hipStream_t s);

// ---- derivative of the hold-out error (k_grad.hip)
hipError_t launch_trmv_interp(int64_t d, int nmat, int M, int q, int c,
                              int64_t ldz, const double* theta_t,
                              const double* w_dev, const double* X, double* Out,
                              hipStream_t s);
hipError_t launch_grad_dot(int64_t d, int nmat, int q, int c, int64_t ldz,
                           const double* x1, const double* y1,
                           const double* x2, const double* y2,
                           const double* lam_dev, const HoldoutNorm& hn,
                           double* partial, double* dlog, int* flags,
                           hipStream_t s);

// ---- accuracy diagnostics (k_nrmse.hip)
// part: tri(ceil(d/128)) * nmat * 4 doubles.
hipError_t launch_factor_nrmse(int64_t d, int nmat, const double* Lhat,
                               const double* L, double* part, double* out,
                               hipStream_t s);
hipError_t launch_holdout_nrmse(const FoldSplit& fs, int c, int q,
                                const double* Y, int64_t ldy,
                                const double* err, double* nrmse,
                                hipStream_t s);

}  // namespace pichol
