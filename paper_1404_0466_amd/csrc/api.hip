// C-ABI of the piCholesky library (declared in include/pichol.h): argument
// validation, workspace layout, host-side FP64 set-up (the pseudo-inverse of
// the observation matrix, lambda scaling) and the order of kernel launches.
#include <math.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "api_internal.hpp"
#include "kernels.hpp"
#include "pichol.h"

namespace pichol {

static thread_local std::string g_last_error;

hipError_t record_hip_error_code(hipError_t e) {
  if (e != hipSuccess) g_last_error = hipGetErrorString(e);
  return e;
}

pichol_status hip_status(hipError_t e) {
  if (e == hipSuccess) return PICHOL_OK;
  record_hip_error_code(e);
  return PICHOL_ERR_HIP;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static std::atomic<int> g_opt_lookahead{0};
int option_lookahead() { return g_opt_lookahead.load(); }
static std::atomic<int> g_opt_group{4};
int option_panel_group() { return g_opt_group.load(); }
static std::atomic<int> g_opt_solve{0};
int option_solve_form() { return g_opt_solve.load(); }

// ---------------------------------------------------------------- profiling
struct ProfState {
  std::mutex mu;
  bool on = false;
  int cap = 0, used = 0;
  std::vector<hipEvent_t> ev;       // 2 per slot
  std::vector<const char*> name;    // per slot
  std::vector<std::string> names_out;
};
static ProfState g_prof;
bool profiling_on() { return g_prof.on; }

ProfScope::ProfScope(const char* n, hipStream_t s) : name(n), stream(s), slot(-1) {
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (!g_prof.on || g_prof.used >= g_prof.cap) return;
  slot = g_prof.used++;
  g_prof.name[slot] = n;
  (void)hipEventRecord(g_prof.ev[2 * slot], s);
}

ProfScope::~ProfScope() {
  if (slot < 0) return;
  (void)hipEventRecord(g_prof.ev[2 * slot + 1], stream);
}

static void prof_destroy() {
  for (hipEvent_t e : g_prof.ev) (void)hipEventDestroy(e);
  g_prof.ev.clear();
  g_prof.name.clear();
  g_prof.cap = g_prof.used = 0;
  g_prof.on = false;
}

// Householder QR of V (g x m, m <= g) and P = V^+ = R^{-1} Q^T (m x g).
// Returns false when V is rank deficient.
static bool pseudo_inverse(int g, int m, const double* V, double* P) {
  std::vector<double> A(V, V + (size_t)g * m);  // row-major g x m
  std::vector<double> Qt((size_t)g * g, 0.0);   // accumulates H_m..H_1
  for (int i = 0; i < g; ++i) Qt[(size_t)i * g + i] = 1.0;
  std::vector<double> v(g);
  for (int j = 0; j < m; ++j) {
    double norm = 0.0;
    for (int i = j; i < g; ++i) norm += A[(size_t)i * m + j] * A[(size_t)i * m + j];
    norm = sqrt(norm);
    if (!(norm > 0.0)) return false;
    const double alpha = A[(size_t)j * m + j] > 0 ? -norm : norm;
    for (int i = 0; i < g; ++i) v[i] = 0.0;
    for (int i = j; i < g; ++i) v[i] = A[(size_t)i * m + j];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < g; ++i) vv += v[i] * v[i];
    if (!(vv > 0.0)) continue;
    // apply I - 2 v v^T / (v^T v) to the columns of A and of Qt
    for (int c = j; c < m; ++c) {
      double s = 0.0;
      for (int i = j; i < g; ++i) s += v[i] * A[(size_t)i * m + c];
      s = 2.0 * s / vv;
      for (int i = j; i < g; ++i) A[(size_t)i * m + c] -= s * v[i];
    }
    for (int c = 0; c < g; ++c) {
      double s = 0.0;
      for (int i = j; i < g; ++i) s += v[i] * Qt[(size_t)i * g + c];
      s = 2.0 * s / vv;
      for (int i = j; i < g; ++i) Qt[(size_t)i * g + c] -= s * v[i];
    }
  }
  // R = A[0:m, 0:m] (upper), P = R^{-1} Qt[0:m, :]
  for (int c = 0; c < g; ++c) {
    for (int i = m - 1; i >= 0; --i) {
      double s = Qt[(size_t)i * g + c];
      for (int k = i + 1; k < m; ++k) s -= A[(size_t)i * m + k] * P[(size_t)k * g + c];
      const double rii = A[(size_t)i * m + i];
      if (!(fabs(rii) > 0.0)) return false;
      P[(size_t)i * g + c] = s / rii;
    }
  }
  return true;
}

bool fold_split(int64_t n, int k, int normalize, FoldSplit* fs) {
  if (k < 2 || k > 64 || n < k) return false;
  memset(fs, 0, sizeof(*fs));
  fs->k = k;
  const int64_t base = n / k, extra = n % k;
  fs->start[0] = 0;
  for (int f = 0; f < k; ++f) {
    fs->start[f + 1] = fs->start[f] + base + (f < extra ? 1 : 0);
    const int64_t ntr = n - (fs->start[f + 1] - fs->start[f]);
    fs->scale[f] = normalize ? 1.0 / (double)ntr : 1.0;
  }
  return true;
}

bool precision_ok(int32_t precision) {
  return precision == PICHOL_PREC_FP64 || precision == PICHOL_PREC_MIXED;
}

bool problem_ok(const pichol_problem* p) {
  return p && p->n >= 1 && p->d >= 1 && p->c >= 1 && p->k >= 2 && p->k <= 64 &&
         p->n >= p->k && p->ldx >= p->d && p->ldy >= p->c && p->q >= 1 &&
         p->g >= 1 && p->g <= 32 && p->r >= 0 && p->r <= 7 && p->r < p->g &&
         precision_ok(p->precision) && p->refine >= 0 &&
         p->refine <= PICHOL_MAX_REFINE && (p->basis == 0 || p->basis == 1);
}

bool samples_ok(const double* lam, int g) {
  for (int s = 0; s < g; ++s) {
    if (!isfinite(lam[s])) return false;
    for (int t = 0; t < s; ++t)
      if (lam[t] == lam[s]) return false;
  }
  return true;
}

// The variable of the fitted polynomials: lambda / lam_ref (basis 0) or
// log(lambda / lam_ref) (basis 1).
double basis_var(double lam, double lam_ref, int basis) {
  return basis ? log(lam / lam_ref) : lam / lam_ref;
}

bool basis_ok(int basis, const double* lam, int n) {
  if (basis == 0) return true;
  if (basis != 1) return false;
  for (int i = 0; i < n; ++i)
    if (!(lam[i] > 0.0)) return false;
  return true;
}

bool fit_coef(int g, int r, const double* lam_s, double lam_ref, int basis,
              FitCoef* fc) {
  const int m = r + 1;
  memset(fc, 0, sizeof(*fc));
  fc->g = g;
  fc->m = m;
  std::vector<double> V((size_t)g * m), P((size_t)m * g);
  for (int s = 0; s < g; ++s) {
    const double tau = basis_var(lam_s[s], lam_ref, basis);
    if (!isfinite(tau)) return false;
    double pw = 1.0;
    for (int j = 0; j < m; ++j) {
      V[(size_t)s * m + j] = pw;
      pw *= tau;
    }
  }
  if (!pseudo_inverse(g, m, V.data(), P.data())) return false;
  for (int j = 0; j < m; ++j)
    for (int s = 0; s < g; ++s) fc->P[j][s] = P[(size_t)j * g + s];
  return true;
}

// Workspace layout of the pipeline calls.
struct Layout {
  int64_t d, nt, dp, S, ldz;
  size_t G, C, yy, H, B, dpart, region;  // byte offsets
  // interpolated region
  size_t i_lam, i_tau, i_L, i_linv, i_th, i_tht, i_Z, i_X, i_part, i_dinv,
      i_end;
  // exact region
  size_t e_lam, e_L, e_linv, e_Z, e_X, e_part, e_end;
  // refinement scratch (full-tile H_f and the correction slab), appended to
  // each method's region when refine > 0
  size_t i_rH, i_rZ, i_lamg, e_rH, e_rZ;
  // gradient scratch (pichol_cv_interp_grad / pichol_cv_exact_grad): the
  // adjoint right-hand sides, four transposed products, plane weights, a
  // zero shift and per-tile partial sums
  size_t i_gS, i_ga1, i_gb1, i_ga2, i_gb2, i_gw, i_gzero, i_gpart, i_gend;
  size_t e_gS, e_gzero, e_gpart, e_gend;
};

static Layout layout_of(const pichol_problem* p) {
  Layout L;
  L.d = p->d;
  L.nt = ntiles_of(p->d);
  L.dp = L.nt * NB;
  L.S = packed_elems_of(p->d);
  L.ldz = ((int64_t)p->q * p->c + NB - 1) / NB * NB;
  const size_t k = (size_t)p->k, dbl = sizeof(double);
  size_t o = 0;
  L.G = o; o += align256(k * L.dp * L.dp * dbl);
  L.C = o; o += align256(k * L.dp * p->c * dbl);
  L.yy = o; o += align256(k * dbl);
  L.H = o; o += align256(k * L.S * dbl);
  L.B = o; o += align256(k * L.dp * p->c * dbl);
  {
    // partial sums of the direct hold-out residual (pichol_cv,
    // pichol_exact_cv)
    FoldSplit fs;
    fold_split(p->n, p->k, p->normalize, &fs);
    L.dpart = o;
    o += align256(k * (size_t)holdout_direct_rowblocks(fs) * L.ldz * dbl);
  }
  L.region = o;
  const size_t g = (size_t)p->g, q = (size_t)p->q, M = (size_t)p->r + 1;
  size_t a = o;
  L.i_lam = a; a += align256(g * dbl);
  L.i_tau = a; a += align256(q * dbl);
  L.i_L = a; a += align256(k * g * L.S * dbl);
  L.i_linv = a; a += align256(k * g * NB2 * dbl);
  L.i_th = a; a += align256(k * M * L.S * dbl);
  L.i_tht = a; a += align256(k * M * L.S * dbl);
  L.i_Z = a; a += align256(k * L.dp * L.ldz * dbl);
  L.i_X = a; a += align256(k * L.dp * L.ldz * dbl);
  L.i_part = a; a += align256(k * L.nt * HOLDOUT_KSPLIT * L.ldz * dbl);
  L.i_dinv = a; a += align256(k * q * L.nt * NB2 * dbl);
  L.i_lamg = a; a += align256(q * dbl);
  const size_t rH = p->refine > 0 ? align256(k * L.dp * L.dp * dbl) : 0;
  const size_t rZ = p->refine > 0 ? align256(k * L.dp * L.ldz * dbl) : 0;
  L.i_rH = a; a += rH;
  L.i_rZ = a; a += rZ;
  L.i_end = a;
  const size_t slab = align256(k * L.dp * L.ldz * dbl);
  L.i_gS = a; a += slab;
  L.i_ga1 = a; a += slab;
  L.i_gb1 = a; a += slab;
  L.i_ga2 = a; a += slab;
  L.i_gb2 = a; a += slab;
  L.i_gw = a; a += align256(2 * 8 * q * dbl);
  L.i_gzero = a; a += align256(q * dbl);
  L.i_gpart = a; a += align256(k * L.nt * q * dbl);
  L.i_gend = a;
  a = o;
  L.e_lam = a; a += align256(q * dbl);
  L.e_L = a; a += align256(k * q * L.S * dbl);
  L.e_linv = a; a += align256(k * q * L.nt * NB2 * dbl);  // every diagonal tile
  L.e_Z = a; a += align256(k * L.dp * L.ldz * dbl);
  L.e_X = a; a += align256(k * L.dp * L.ldz * dbl);
  L.e_part = a; a += align256(k * L.nt * HOLDOUT_KSPLIT * L.ldz * dbl);
  L.e_rH = a; a += rH;
  L.e_rZ = a; a += rZ;
  L.e_end = a;
  L.e_gS = a; a += slab;
  L.e_gzero = a; a += align256(q * dbl);
  L.e_gpart = a; a += align256(k * L.nt * q * dbl);
  L.e_gend = a;
  return L;
}

template <typename T>
static T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

void holdout_norm(const pichol_problem* p, HoldoutNorm* hn) {
  FoldSplit fs;
  fold_split(p->n, p->k, p->normalize, &fs);
  memset(hn, 0, sizeof(*hn));
  hn->nmat = p->k;
  for (int f = 0; f < p->k; ++f)
    hn->count[f] = (double)(fs.start[f + 1] - fs.start[f]) * (double)p->c;
}

hipError_t upload_tau(const double* lam, int nlam, double lam_ref, int basis,
                      double* dst, hipStream_t stream) {
  std::vector<double> tau(nlam);
  for (int t = 0; t < nlam; ++t) tau[t] = basis_var(lam[t], lam_ref, basis);
  return launch_store_doubles(tau.data(), nlam, dst, stream);
}

}  // namespace pichol

using namespace pichol;

// Scratch of pichol_holdout_noalloc: the partial sums of the hold-out
// product, in a file-scope device array instead of a caller's workspace.
// Each device holds its own copy; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[PICHOL_HOLDOUT_SCRATCH_BYTES /
                                                sizeof(double)];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static hipError_t scratch_address(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// An argument error with a message for pichol_last_error.
static pichol_status arg_error(pichol_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

extern "C" {

int64_t pichol_packed_elems(int64_t d) { return packed_elems_of(d); }
int64_t pichol_padded_order(int64_t d) { return d < 1 ? 0 : ntiles_of(d) * NB; }
int64_t pichol_slab_cols(int64_t q, int64_t c) {
  return (q < 1 || c < 1) ? 0 : (q * c + NB - 1) / NB * NB;
}

const char* pichol_status_string(pichol_status s) {
  switch (s) {
    case PICHOL_OK: return "ok";
    case PICHOL_ERR_ARG: return "invalid argument";
    case PICHOL_ERR_WORKSPACE: return "workspace missing or too small";
    case PICHOL_ERR_HIP: return "HIP runtime error";
    case PICHOL_ERR_NOT_PD: return "a shifted matrix is not positive definite";
    case PICHOL_ERR_DATA: return "non-finite result or non-positive interpolated pivot";
  }
  return "unknown status";
}

const char* pichol_last_error(void) { return g_last_error.c_str(); }

pichol_status pichol_set_option(int32_t option, int32_t value) {
  switch (option) {
    case PICHOL_OPT_LOOKAHEAD:
      if (value != 0 && value != 1) return PICHOL_ERR_ARG;
      g_opt_lookahead.store(value);
      return PICHOL_OK;
    case PICHOL_OPT_PANEL_GROUP:
      if (value < 1 || value > 8) return PICHOL_ERR_ARG;
      g_opt_group.store(value);
      return PICHOL_OK;
    case PICHOL_OPT_SOLVE_FORM:
      if (value < 0 || value > 2) return PICHOL_ERR_ARG;
      g_opt_solve.store(value);
      return PICHOL_OK;
  }
  return PICHOL_ERR_ARG;
}

int32_t pichol_get_option(int32_t option) {
  switch (option) {
    case PICHOL_OPT_LOOKAHEAD: return g_opt_lookahead.load();
    case PICHOL_OPT_PANEL_GROUP: return g_opt_group.load();
    case PICHOL_OPT_SOLVE_FORM: return g_opt_solve.load();
  }
  return -1;
}

pichol_status pichol_profile_start(int32_t capacity) {
  if (capacity < 1) return PICHOL_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  prof_destroy();
  g_prof.ev.resize(2 * (size_t)capacity, nullptr);
  for (auto& e : g_prof.ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      e = nullptr;
      prof_destroy();
      return hip_status(r);
    }
  }
  g_prof.name.assign(capacity, nullptr);
  g_prof.cap = capacity;
  g_prof.used = 0;
  g_prof.on = true;
  return PICHOL_OK;
}

pichol_status pichol_profile_stop(void) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = false;
  return PICHOL_OK;
}

int32_t pichol_profile_summary(int32_t max, const char** names,
                               int64_t* launches, double* total_ms) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  std::map<std::string, std::pair<int64_t, double>> agg;
  for (int sl = 0; sl < g_prof.used; ++sl) {
    float ms = 0.0f;
    if (hipEventSynchronize(g_prof.ev[2 * sl + 1]) != hipSuccess) return -1;
    if (hipEventElapsedTime(&ms, g_prof.ev[2 * sl], g_prof.ev[2 * sl + 1]) != hipSuccess)
      return -1;
    auto& a = agg[g_prof.name[sl]];
    a.first += 1;
    a.second += ms;
  }
  g_prof.names_out.clear();
  int32_t i = 0;
  for (auto& kv : agg) {
    if (i < max) {
      g_prof.names_out.push_back(kv.first);
      if (launches) launches[i] = kv.second.first;
      if (total_ms) total_ms[i] = kv.second.second;
    }
    ++i;
  }
  if (names)
    for (int32_t j = 0; j < (int32_t)g_prof.names_out.size(); ++j)
      names[j] = g_prof.names_out[j].c_str();
  return i;
}

pichol_status pichol_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  prof_destroy();
  g_prof.names_out.clear();
  return PICHOL_OK;
}

pichol_status pichol_pack(int64_t d, int32_t nmat, const double* A, int64_t lda,
                          double* P, hipStream_t stream) {
  if (d < 1 || nmat < 1 || !A || !P || lda < d) return PICHOL_ERR_ARG;
  return hip_status(launch_pack(d, nmat, A, lda, P, stream));
}

pichol_status pichol_unpack(int64_t d, int32_t nmat, const double* P, double* A,
                            int64_t lda, hipStream_t stream) {
  if (d < 1 || nmat < 1 || !A || !P || lda < d) return PICHOL_ERR_ARG;
  return hip_status(launch_unpack(d, nmat, P, A, lda, stream));
}

pichol_status pichol_gram(const pichol_problem* p, const double* X,
                          const double* Y, double* G, double* C, double* yy,
                          double* H, double* B, hipStream_t stream) {
  if (!p || p->n < 1 || p->d < 1 || p->c < 1 || p->ldx < p->d || p->ldy < p->c)
    return PICHOL_ERR_ARG;
  if (!X || !Y || !G || !C || !yy || !H || !B) return PICHOL_ERR_ARG;
  FoldSplit fs;
  if (!fold_split(p->n, p->k, p->normalize, &fs)) return PICHOL_ERR_ARG;
  return hip_status(launch_gram(X, p->ldx, Y, p->ldy, p->d, p->c, fs, G, C, yy,
                                H, B, stream));
}

size_t pichol_factor_nrmse_workspace(int64_t d, int32_t nmat) {
  if (d < 1 || nmat < 1) return 0;
  return align256((size_t)tri(ntiles_of(d)) * nmat * 4 * sizeof(double));
}

pichol_status pichol_factor_nrmse(int64_t d, int32_t nmat, const double* Lhat,
                                  const double* L, double* out, void* ws,
                                  size_t ws_bytes, hipStream_t stream) {
  if (d < 1 || nmat < 1 || !Lhat || !L || !out) return PICHOL_ERR_ARG;
  if (!ws || ws_bytes < pichol_factor_nrmse_workspace(d, nmat))
    return PICHOL_ERR_WORKSPACE;
  return hip_status(launch_factor_nrmse(d, nmat, Lhat, L, at<double>(ws, 0),
                                        out, stream));
}

pichol_status pichol_holdout_nrmse(const pichol_problem* p, const double* Y,
                                   const double* err, double* nrmse,
                                   hipStream_t stream) {
  if (!problem_ok(p) || !Y || !err || !nrmse) return PICHOL_ERR_ARG;
  FoldSplit fs;
  if (!fold_split(p->n, p->k, p->normalize, &fs)) return PICHOL_ERR_ARG;
  return hip_status(launch_holdout_nrmse(fs, (int)p->c, p->q, Y, p->ldy, err,
                                         nrmse, stream));
}

size_t pichol_potrf_workspace(int32_t nmat, int32_t nshift) {
  if (nmat < 1 || nshift < 1) return 0;
  return align256((size_t)nshift * sizeof(double)) +
         align256((size_t)nmat * nshift * NB2 * sizeof(double));
}

pichol_status pichol_potrf_shifted_batched(int64_t d, int32_t nmat,
                                           const double* H, int32_t nshift,
                                           const double* lam, double* L,
                                           int32_t* info, void* ws,
                                           size_t ws_bytes, int32_t precision,
                                           hipStream_t stream) {
  if (d < 1 || nmat < 1 || nshift < 1 || !H || !lam || !L || !info ||
      !precision_ok(precision))
    return PICHOL_ERR_ARG;
  for (int s = 0; s < nshift; ++s)
    if (!isfinite(lam[s])) return PICHOL_ERR_ARG;
  if (!ws || ws_bytes < pichol_potrf_workspace(nmat, nshift))
    return PICHOL_ERR_WORKSPACE;
  double* lam_dev = at<double>(ws, 0);
  double* linv = at<double>(ws, align256((size_t)nshift * sizeof(double)));
  hipError_t e = launch_store_doubles(lam, nshift, lam_dev, stream);
  if (e != hipSuccess) return hip_status(e);
  const ShiftSrc src{H, nshift, lam_dev, nmat};
  return hip_status(launch_potrf_blocked(d, nmat * nshift, src, L, info, linv,
                                         0, precision == PICHOL_PREC_MIXED,
                                         option_lookahead(), 0, stream));
}

pichol_status pichol_fit(int64_t d, int32_t nmat, int32_t g, int32_t r,
                         const double* lam_s, double lam_ref, const double* L,
                         double* theta, double* theta_t, hipStream_t stream) {
  if (d < 1 || nmat < 1 || g < 1 || g > 32 || r < 0 || r > 7 || r >= g ||
      !lam_s || !L || !theta || !(lam_ref > 0.0) || !isfinite(lam_ref))
    return PICHOL_ERR_ARG;
  if (!samples_ok(lam_s, g)) return PICHOL_ERR_ARG;
  FitCoef fc;
  if (!fit_coef(g, r, lam_s, lam_ref, 0, &fc)) return PICHOL_ERR_ARG;
  return hip_status(launch_fit(d, nmat, fc, L, theta, theta_t, stream));
}

size_t pichol_lambda_workspace(int32_t nlam) {
  return nlam < 1 ? 0 : align256((size_t)nlam * sizeof(double));
}

// [scaled lambdas | inverses | second slab]
static size_t solve_inv_bytes(int64_t d, int32_t nmat, int32_t q) {
  return align256((size_t)nmat * q * ntiles_of(d) * NB2 * sizeof(double));
}

size_t pichol_solve_interp_workspace(int64_t d, int32_t nmat, int32_t q,
                                     int32_t c) {
  if (d < 1 || nmat < 1 || q < 1 || c < 1) return 0;
  return pichol_lambda_workspace(q) + solve_inv_bytes(d, nmat, q) +
         align256((size_t)nmat * ntiles_of(d) * NB * pichol_slab_cols(q, c) *
                  sizeof(double));
}


pichol_status pichol_eval(int64_t d, int32_t nmat, int32_t r,
                          const double* theta, int32_t nlam, const double* lam,
                          double lam_ref, double* Lhat, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
  if (d < 1 || nmat < 1 || r < 0 || r > 7 || nlam < 1 || !theta || !lam ||
      !Lhat || !(lam_ref > 0.0) || !isfinite(lam_ref))
    return PICHOL_ERR_ARG;
  if (!ws || ws_bytes < pichol_lambda_workspace(nlam)) return PICHOL_ERR_WORKSPACE;
  double* tau = at<double>(ws, 0);
  hipError_t e = upload_tau(lam, nlam, lam_ref, 0, tau, stream);
  if (e != hipSuccess) return hip_status(e);
  return hip_status(launch_eval(d, nmat, r + 1, theta, nlam, tau, Lhat, stream));
}

pichol_status pichol_solve_interp(int64_t d, int32_t nmat, int32_t c, int32_t r,
                                  const double* theta, const double* theta_t,
                                  const double* B, int32_t q, const double* lam,
                                  double lam_ref, double* Z, int32_t* flags,
                                  void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
  if (d < 1 || nmat < 1 || c < 1 || r < 0 || r > 7 || q < 1 || !theta ||
      !theta_t || !B || !lam || !Z || !flags || !(lam_ref > 0.0) ||
      !isfinite(lam_ref))
    return PICHOL_ERR_ARG;
  if (!ws || ws_bytes < pichol_solve_interp_workspace(d, nmat, q, c))
    return PICHOL_ERR_WORKSPACE;
  const int64_t ldz = pichol_slab_cols(q, c);
  double* tau = at<double>(ws, 0);
  double* dinv = at<double>(ws, pichol_lambda_workspace(q));
  double* X = at<double>(ws, pichol_lambda_workspace(q) +
                                 solve_inv_bytes(d, nmat, q));
  hipError_t e = upload_tau(lam, q, lam_ref, 0, tau, stream);
  if (e == hipSuccess) e = launch_slab_init(d, nmat, q, c, ldz, B, Z, flags, stream);
  if (e == hipSuccess)
    e = launch_solve_interp(d, nmat, c, r + 1, theta, theta_t, q, tau, ldz, Z,
                            X, flags, dinv, 1, stream);
  return hip_status(e);
}

pichol_status pichol_solve_factors(int64_t d, int32_t nmat, int32_t nper,
                                   int32_t c, const double* L, const double* B,
                                   double* Z, int32_t* flags,
                                   hipStream_t stream) {
  if (d < 1 || nmat < 1 || nper < 1 || c < 1 || !L || !B || !Z || !flags)
    return PICHOL_ERR_ARG;
  const int64_t ldz = pichol_slab_cols(nper, c);
  hipError_t e = launch_slab_init(d, nmat, nper, c, ldz, B, Z, flags, stream);
  if (e == hipSuccess)
    e = launch_solve_factors(d, nmat, nper, c, L, ldz, Z, flags, nullptr,
                             nullptr, stream);
  return hip_status(e);
}

size_t pichol_holdout_workspace(int64_t d, int32_t nmat, int32_t q, int32_t c) {
  if (d < 1 || nmat < 1 || q < 1 || c < 1) return 0;
  return align256((size_t)nmat * ntiles_of(d) * HOLDOUT_KSPLIT *
                  pichol_slab_cols(q, c) * sizeof(double));
}

pichol_status pichol_holdout(int64_t d, int32_t nmat, int32_t c, int32_t q,
                             const double* Z, const double* G, const double* C,
                             const double* yy, const int64_t* nv, double* err,
                             int32_t* flags, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
  if (d < 1 || nmat < 1 || nmat > 64 || c < 1 || q < 1 || !Z || !G || !C ||
      !yy || !nv || !err || !flags)
    return PICHOL_ERR_ARG;
  if (!ws || ws_bytes < pichol_holdout_workspace(d, nmat, q, c))
    return PICHOL_ERR_WORKSPACE;
  HoldoutNorm hn;
  memset(&hn, 0, sizeof(hn));
  hn.nmat = nmat;
  for (int m = 0; m < nmat; ++m) {
    if (nv[m] < 1) return PICHOL_ERR_ARG;
    hn.count[m] = (double)nv[m] * (double)c;
  }
  return hip_status(launch_holdout(d, nmat, c, q, pichol_slab_cols(q, c), Z, G,
                                   C, yy, hn, static_cast<double*>(ws), err,
                                   flags, stream));
}

pichol_status pichol_holdout_noalloc(int64_t d, int32_t nmat, int32_t c,
                                     int32_t q, const double* Z,
                                     const double* G, const double* C,
                                     const double* yy, const int64_t* nv,
                                     double* err, int32_t* flags,
                                     hipStream_t stream) {
  if (d < 1 || nmat < 1 || nmat > 64 || c < 1 || q < 1 || !Z || !G || !C ||
      !yy || !nv || !err || !flags)
    return arg_error(PICHOL_ERR_ARG, "pichol_holdout_noalloc: invalid argument");
  const size_t need = pichol_holdout_workspace(d, nmat, q, c);
  if (need > PICHOL_HOLDOUT_SCRATCH_BYTES)
    return arg_error(PICHOL_ERR_WORKSPACE,
                "pichol_holdout_noalloc: the partial sums need " +
                    std::to_string(need) + " bytes, more than the " +
                    std::to_string((size_t)PICHOL_HOLDOUT_SCRATCH_BYTES) +
                    " bytes of the static scratch (use pichol_holdout)");
  HoldoutNorm hn;
  memset(&hn, 0, sizeof(hn));
  hn.nmat = nmat;
  for (int m = 0; m < nmat; ++m) {
    if (nv[m] < 1)
      return arg_error(PICHOL_ERR_ARG, "pichol_holdout_noalloc: nv[m] < 1");
    hn.count[m] = (double)nv[m] * (double)c;
  }
  double* part = nullptr;
  hipError_t e = scratch_address(&part);
  if (e != hipSuccess) return hip_status(e);
  // every partial sum the final reduction reads is written by the partial
  // kernel (ranges above the diagonal and padding columns as zeros), so the
  // scratch needs no clearing between calls
  return hip_status(launch_holdout(d, nmat, c, q, pichol_slab_cols(q, c), Z, G,
                                   C, yy, hn, part, err, flags, stream));
}

size_t pichol_holdout_direct_workspace(const pichol_problem* p) {
  if (!p || p->n < 1 || p->q < 1 || p->c < 1) return 0;
  FoldSplit fs;
  if (!fold_split(p->n, p->k, p->normalize, &fs)) return 0;
  return align256((size_t)p->k * holdout_direct_rowblocks(fs) *
                  pichol_slab_cols(p->q, p->c) * sizeof(double));
}

pichol_status pichol_holdout_direct(const pichol_problem* p, const double* X,
                                    const double* Y, const double* Z,
                                    double* err, int32_t* flags, void* ws,
                                    size_t ws_bytes, hipStream_t stream) {
  if (!p || p->n < 1 || p->d < 1 || p->c < 1 || p->q < 1 || p->ldx < p->d ||
      p->ldy < p->c || !X || !Y || !Z || !err || !flags)
    return PICHOL_ERR_ARG;
  FoldSplit fs;
  if (!fold_split(p->n, p->k, p->normalize, &fs)) return PICHOL_ERR_ARG;
  if (!ws || ws_bytes < pichol_holdout_direct_workspace(p))
    return PICHOL_ERR_WORKSPACE;
  HoldoutNorm hn;
  holdout_norm(p, &hn);
  return hip_status(launch_holdout_direct(
      p->d, p->k, (int)p->c, p->q, pichol_slab_cols(p->q, p->c), Z, X, p->ldx,
      Y, p->ldy, fs, hn, static_cast<double*>(ws), err, flags, 0, stream));
}

pichol_status pichol_slab_to_weights(int64_t d, int32_t nmat, int32_t q,
                                     int32_t c, const double* Z, double* W,
                                     hipStream_t stream) {
  if (d < 1 || nmat < 1 || q < 1 || c < 1 || !Z || !W) return PICHOL_ERR_ARG;
  return hip_status(launch_slab_to_weights(d, nmat, q, c, pichol_slab_cols(q, c),
                                           Z, W, stream));
}

// PINRMSE workspace: the exact pipeline's layout at the g samples, then the
// sample errors and the scaled grid values.
static size_t pinrmse_es(const pichol_problem* p) {
  pichol_problem ps = *p;
  ps.q = p->g;
  ps.refine = 0;
  return layout_of(&ps).e_end;
}
static size_t pinrmse_tau(const pichol_problem* p) {
  return pinrmse_es(p) + align256((size_t)p->k * p->g * sizeof(double));
}
static size_t pinrmse_end(const pichol_problem* p) {
  return pinrmse_tau(p) + align256((size_t)p->q * sizeof(double));
}

pichol_status pichol_workspace_size(const pichol_problem* p, int32_t methods,
                                    size_t* bytes) {
  if (!bytes || !problem_ok(p) ||
      (methods & ~(PICHOL_METHOD_INTERP | PICHOL_METHOD_EXACT |
                   PICHOL_METHOD_GRAD | PICHOL_METHOD_PINRMSE)) ||
      !(methods & (PICHOL_METHOD_INTERP | PICHOL_METHOD_EXACT |
                   PICHOL_METHOD_PINRMSE)))
    return PICHOL_ERR_ARG;
  if (methods & PICHOL_METHOD_PINRMSE) {
    size_t pe = pinrmse_end(p);
    if ((methods & ~PICHOL_METHOD_PINRMSE) == 0) {
      *bytes = pe;
      return PICHOL_OK;
    }
    size_t rest = 0;
    pichol_status st = pichol_workspace_size(p, methods & ~PICHOL_METHOD_PINRMSE,
                                             &rest);
    if (st != PICHOL_OK) return st;
    *bytes = pe > rest ? pe : rest;
    return PICHOL_OK;
  }
  const Layout L = layout_of(p);
  const bool grad = (methods & PICHOL_METHOD_GRAD) != 0;
  size_t end = L.region;
  const size_t ie = grad ? L.i_gend : L.i_end, ee = grad ? L.e_gend : L.e_end;
  if (methods & PICHOL_METHOD_INTERP) end = end > ie ? end : ie;
  if (methods & PICHOL_METHOD_EXACT) end = end > ee ? end : ee;
  *bytes = end;
  return PICHOL_OK;
}

pichol_status pichol_cv_gram(const pichol_problem* p, const double* X,
                             const double* Y, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
  if (!problem_ok(p) || !X || !Y) return PICHOL_ERR_ARG;
  const Layout L = layout_of(p);
  if (!ws || ws_bytes < L.region) return PICHOL_ERR_WORKSPACE;
  return pichol_gram(p, X, Y, at<double>(ws, L.G), at<double>(ws, L.C),
                     at<double>(ws, L.yy), at<double>(ws, L.H),
                     at<double>(ws, L.B), stream);
}

// Second stream of the interpolated pipeline (default priority, created
// once per device with two events).  While the last kLateColumns columns of
// the sample factors are factored (short, latency-bound launches that leave
// most of the GPU idle), it fits the columns already finished, inverts
// their interpolated diagonal blocks and runs the forward solve steps that
// need only those columns.
namespace {
constexpr int kLateColumns = 12;
struct OverlapStream {
  bool ready = false;
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, done = nullptr;
};
std::mutex g_overlap_mu;
OverlapStream g_overlap[64];

OverlapStream* overlap_stream() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  OverlapStream& os = g_overlap[dev];
  if (!os.ready) {
    // each handle is created once: a call that failed part-way keeps what it
    // made and the next call creates only the rest
    if (!os.stream &&
        hipStreamCreateWithFlags(&os.stream, hipStreamNonBlocking) != hipSuccess) {
      os.stream = nullptr;
      return nullptr;
    }
    if (!os.start &&
        hipEventCreateWithFlags(&os.start, hipEventDisableTiming) != hipSuccess) {
      os.start = nullptr;
      return nullptr;
    }
    if (!os.done &&
        hipEventCreateWithFlags(&os.done, hipEventDisableTiming) != hipSuccess) {
      os.done = nullptr;
      return nullptr;
    }
    os.ready = true;
  }
  return &os;
}

// The early part of the fit and of the diagonal-block inverses, forked off
// the caller's stream once column cols-1 of every sample factor is final,
// and (fwd > 0, the per-lambda solve form) the forward solve steps
// 0 .. fwd-1, which read only those columns' coefficients and inverses.
struct EarlyFit {
  OverlapStream* os;
  hipStream_t main;
  int64_t d;
  int k, q, M, cols, c;
  const FitCoef* fc;
  const double* Lf;
  double *th, *tht, *dinv;
  const double* tau;
  int* flags;
  int fwd;
  int64_t ldz;
  double *Z, *X;
};

hipError_t early_fit(void* ctx) {
  const EarlyFit& c = *static_cast<const EarlyFit*>(ctx);
  hipError_t e = hipEventRecord(c.os->start, c.main);
  if (e == hipSuccess) e = hipStreamWaitEvent(c.os->stream, c.os->start, 0);
  if (e != hipSuccess) return e;
  e = launch_fit_cols(c.d, c.k, *c.fc, c.Lf, c.th, c.tht, 0, c.cols,
                      c.os->stream);
  if (e == hipSuccess)
    e = launch_diag_inv(c.d, c.k, c.M, c.th, c.q, c.tau, c.dinv, c.flags, 0,
                        c.cols, c.os->stream);
  if (e == hipSuccess && c.fwd > 0)
    e = launch_solve_fwd(c.d, c.k, c.c, c.M, c.th, c.q, c.tau, c.ldz, c.Z, c.X,
                         c.dinv, 0, c.fwd, c.os->stream);
  // the caller's stream waits for this event before it needs the results,
  // so it is recorded even after a failed launch
  const hipError_t r = hipEventRecord(c.os->done, c.os->stream);
  return e != hipSuccess ? e : r;
}
}  // namespace

pichol_status pichol_cv_interp(const pichol_problem* p, const double* lam_s,
                               const double* lam_grid, double lam_ref, void* ws,
                               size_t ws_bytes, double* err, double* W,
                               int32_t* info, int32_t* flags,
                               hipStream_t stream) {
  if (!problem_ok(p) || !lam_s || !lam_grid || !err || !info || !flags ||
      !(lam_ref > 0.0) || !isfinite(lam_ref))
    return PICHOL_ERR_ARG;
  if (!samples_ok(lam_s, p->g)) return PICHOL_ERR_ARG;
  for (int t = 0; t < p->q; ++t)
    if (!isfinite(lam_grid[t])) return PICHOL_ERR_ARG;
  const Layout L = layout_of(p);
  if (!ws || ws_bytes < L.i_end) return PICHOL_ERR_WORKSPACE;
  FitCoef fc;
  if (!basis_ok(p->basis, lam_s, p->g) || !basis_ok(p->basis, lam_grid, p->q))
    return PICHOL_ERR_ARG;
  if (!fit_coef(p->g, p->r, lam_s, lam_ref, p->basis, &fc)) return PICHOL_ERR_ARG;
  HoldoutNorm hn;
  holdout_norm(p, &hn);
  const int k = p->k, g = p->g, q = p->q, c = (int)p->c, M = p->r + 1;
  double* lam_dev = at<double>(ws, L.i_lam);
  double* tau = at<double>(ws, L.i_tau);
  double* Lf = at<double>(ws, L.i_L);
  double* th = at<double>(ws, L.i_th);
  double* tht = at<double>(ws, L.i_tht);
  double* Z = at<double>(ws, L.i_Z);
  double* dinv = at<double>(ws, L.i_dinv);
  hipError_t e = launch_store_doubles(lam_s, g, lam_dev, stream);
  if (e == hipSuccess)
    e = upload_tau(lam_grid, q, lam_ref, p->basis, tau, stream);
  // the flags are cleared here, before any diagonal-block inverse can set
  // one of their bits
  if (e == hipSuccess)
    e = launch_slab_init(p->d, k, q, c, L.ldz, at<double>(ws, L.B), Z, flags,
                         stream);
  // columns 0 .. cols-1 are fitted and their diagonal blocks inverted on the
  // second stream while the last columns are still being factored
  const int nt = (int)L.nt;
  // (not under stream capture: the shared second stream would join the
  // caller's capture, and any other call using it meanwhile would land in
  // or break that capture; the results are the same either way)
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (stream && hipStreamIsCapturing(stream, &cap) != hipSuccess)
    cap = hipStreamCaptureStatusActive;  // unknown: do not fork
  std::unique_lock<std::mutex> lk(g_overlap_mu, std::defer_lock);
  OverlapStream* os = nullptr;
  if (nt > kLateColumns && cap == hipStreamCaptureStatusNone) {
    lk.lock();
    os = overlap_stream();
  }
  const int cols = os ? nt - kLateColumns : 0;
  // forward steps 0 .. cols-2 need only the early columns (step i reads
  // column i and the inverse of block i+1)
  const int fwd = (os && solve_form_for(M, q, c, L.ldz, 0) == 2) ? cols - 1 : 0;
  EarlyFit ef{os, stream, p->d, k, q, M, cols, c, &fc, Lf, th, tht, dinv, tau,
              flags, fwd, L.ldz, Z, at<double>(ws, L.i_X)};
  const PanelHook hook{cols - 1, early_fit, &ef};
  if (e == hipSuccess)
    e = launch_potrf_blocked(p->d, k * g,
                             ShiftSrc{at<double>(ws, L.H), g, lam_dev, k}, Lf,
                             info, at<double>(ws, L.i_linv), 0,
                             p->precision == PICHOL_PREC_MIXED,
                             option_lookahead(), 0, stream, os ? &hook : nullptr);
  if (e == hipSuccess)
    e = launch_fit_cols(p->d, k, fc, Lf, th, tht, cols, nt, stream);
  // the late columns' inverses touch nothing the second stream uses (their
  // own blocks; flag bits are set atomically), so they run beside its
  // forward steps
  if (e == hipSuccess)
    e = launch_diag_inv(p->d, k, M, th, q, tau, dinv, flags, cols, nt, stream);
  if (os) {
    // join the second stream (its work was forked by the hook, which ran
    // unless an earlier launch failed)
    const hipError_t j = hipStreamWaitEvent(stream, os->done, 0);
    if (e == hipSuccess) e = j;
  }
  if (e == hipSuccess)
    e = launch_solve_interp(p->d, k, c, M, th, tht, q, tau, L.ldz, Z,
                            at<double>(ws, L.i_X), flags, dinv, 0, stream, fwd);
  if (e == hipSuccess && p->refine > 0) {
    // Residual correction against H_f + lambda_t I; the correction solves
    // reuse the inverted diagonal blocks of the interpolated factors.
    double* Hf = at<double>(ws, L.i_rH);
    double* D = at<double>(ws, L.i_rZ);
    double* lamg = at<double>(ws, L.i_lamg);
    FoldSplit fs;
    fold_split(p->n, p->k, p->normalize, &fs);
    e = launch_store_doubles(lam_grid, q, lamg, stream);
    if (e == hipSuccess) e = launch_full_h(p->d, fs, at<double>(ws, L.G), Hf, stream);
    for (int it = 0; it < p->refine && e == hipSuccess; ++it) {
      e = launch_residual(p->d, k, q, c, L.ldz, Hf, at<double>(ws, L.B), lamg,
                          Z, D, stream);
      if (e == hipSuccess)
        e = launch_solve_interp(p->d, k, c, M, th, tht, q, tau, L.ldz, D,
                                at<double>(ws, L.i_X), flags,
                                at<double>(ws, L.i_dinv),
                                0, stream);
      if (e == hipSuccess) e = launch_slab_add(p->d, k, L.ldz, D, Z, stream);
    }
  }
  if (e == hipSuccess)
    e = launch_holdout(p->d, k, c, q, L.ldz, Z, at<double>(ws, L.G),
                       at<double>(ws, L.C), at<double>(ws, L.yy), hn,
                       at<double>(ws, L.i_part), err, flags, stream);
  if (e == hipSuccess && W)
    e = launch_slab_to_weights(p->d, k, q, c, L.ldz, Z, W, stream);
  return hip_status(e);
}

pichol_status pichol_cv_exact(const pichol_problem* p, const double* lam_grid,
                              void* ws, size_t ws_bytes, double* err, double* W,
                              int32_t* info, int32_t* flags,
                              hipStream_t stream) {
  if (!problem_ok(p) || !lam_grid || !err || !info || !flags)
    return PICHOL_ERR_ARG;
  for (int t = 0; t < p->q; ++t)
    if (!isfinite(lam_grid[t])) return PICHOL_ERR_ARG;
  const Layout L = layout_of(p);
  if (!ws || ws_bytes < L.e_end) return PICHOL_ERR_WORKSPACE;
  HoldoutNorm hn;
  holdout_norm(p, &hn);
  const int k = p->k, q = p->q, c = (int)p->c;
  double* lam_dev = at<double>(ws, L.e_lam);
  double* Lf = at<double>(ws, L.e_L);
  double* Z = at<double>(ws, L.e_Z);
  hipError_t e = launch_store_doubles(lam_grid, q, lam_dev, stream);
  if (e == hipSuccess)
    e = launch_potrf_blocked(p->d, k * q,
                             ShiftSrc{at<double>(ws, L.H), q, lam_dev, k}, Lf,
                             info, at<double>(ws, L.e_linv), 1,
                             p->precision == PICHOL_PREC_MIXED,
                             option_lookahead(), 0, stream);
  if (e == hipSuccess)
    e = launch_slab_init(p->d, k, q, c, L.ldz, at<double>(ws, L.B), Z, flags,
                         stream);
  if (e == hipSuccess)
    e = launch_solve_factors(p->d, k, q, c, Lf, L.ldz, Z, flags,
                             at<double>(ws, L.e_linv), at<double>(ws, L.e_X),
                             stream);
  if (e == hipSuccess && p->refine > 0) {
    double* Hf = at<double>(ws, L.e_rH);
    double* D = at<double>(ws, L.e_rZ);
    FoldSplit fs;
    fold_split(p->n, p->k, p->normalize, &fs);
    e = launch_full_h(p->d, fs, at<double>(ws, L.G), Hf, stream);
    for (int it = 0; it < p->refine && e == hipSuccess; ++it) {
      e = launch_residual(p->d, k, q, c, L.ldz, Hf, at<double>(ws, L.B),
                          lam_dev, Z, D, stream);
      if (e == hipSuccess)
        e = launch_solve_factors(p->d, k, q, c, Lf, L.ldz, D, flags,
                                 at<double>(ws, L.e_linv),
                                 at<double>(ws, L.e_X), stream);
      if (e == hipSuccess) e = launch_slab_add(p->d, k, L.ldz, D, Z, stream);
    }
  }
  if (e == hipSuccess)
    e = launch_holdout(p->d, k, c, q, L.ldz, Z, at<double>(ws, L.G),
                       at<double>(ws, L.C), at<double>(ws, L.yy), hn,
                       at<double>(ws, L.e_part), err, flags, stream);
  if (e == hipSuccess && W)
    e = launch_slab_to_weights(p->d, k, q, c, L.ldz, Z, W, stream);
  return hip_status(e);
}

pichol_status pichol_cv_interp_grad(const pichol_problem* p,
                                    const double* lam_s,
                                    const double* lam_grid, double lam_ref,
                                    void* ws, size_t ws_bytes, double* err,
                                    double* dlog, double* W, int32_t* info,
                                    int32_t* flags, hipStream_t stream) {
  if (!problem_ok(p) || p->refine != 0 || !dlog) return PICHOL_ERR_ARG;
  const Layout L = layout_of(p);
  if (!ws || ws_bytes < L.i_gend) return PICHOL_ERR_WORKSPACE;
  // forward: the piCholesky stage (solutions in the slab, hold-out errors)
  pichol_status st = pichol_cv_interp(p, lam_s, lam_grid, lam_ref, ws, ws_bytes,
                                      err, W, info, flags, stream);
  if (st != PICHOL_OK) return st;
  const int k = p->k, q = p->q, c = (int)p->c, M = p->r + 1;
  double* Z = at<double>(ws, L.i_Z);
  double* Sg = at<double>(ws, L.i_gS);
  double* th_t = at<double>(ws, L.i_tht);
  double* wts = at<double>(ws, L.i_gw);
  // plane weights per lambda: tau^p (value) and p tau^(p-1) / lam_ref
  std::vector<double> w(2 * 8 * (size_t)q, 0.0), zero(q, 0.0);
  for (int t = 0; t < q; ++t) {
    const double tau = basis_var(lam_grid[t], lam_ref, p->basis);
    // d(variable)/d(lambda)
    const double dvar = p->basis ? 1.0 / lam_grid[t] : 1.0 / lam_ref;
    double pw = 1.0, pwm1 = 0.0;  // tau^p, tau^(p-1)
    for (int pp = 0; pp < M; ++pp) {
      w[(size_t)pp * q + t] = pw;
      w[(size_t)(8 + pp) * q + t] = pp == 0 ? 0.0 : (double)pp * pwm1 * dvar;
      pwm1 = pw;
      pw *= tau;
    }
  }
  HoldoutNorm hn;
  holdout_norm(p, &hn);
  double* lamg = at<double>(ws, L.i_lamg);
  hipError_t e = launch_store_doubles(w.data(), 16 * q, wts, stream);
  if (e == hipSuccess)
    e = launch_store_doubles(zero.data(), q, at<double>(ws, L.i_gzero), stream);
  if (e == hipSuccess) e = launch_store_doubles(lam_grid, q, lamg, stream);
  // X_v^T R = C_v - G_v theta for every lambda (a zero shift)
  if (e == hipSuccess)
    e = launch_residual(p->d, k, q, c, L.ldz, at<double>(ws, L.G),
                        at<double>(ws, L.C), at<double>(ws, L.i_gzero), Z, Sg,
                        stream);
  // z = A^{-1} X_v^T R with the stored diagonal-block inverses
  if (e == hipSuccess)
    e = launch_solve_interp(p->d, k, c, M, at<double>(ws, L.i_th), th_t, q,
                            at<double>(ws, L.i_tau), L.ldz, Sg,
                            at<double>(ws, L.i_X), flags,
                            at<double>(ws, L.i_dinv), 0, stream);
  double* a1 = at<double>(ws, L.i_ga1);
  double* b1 = at<double>(ws, L.i_gb1);
  double* a2 = at<double>(ws, L.i_ga2);
  double* b2 = at<double>(ws, L.i_gb2);
  if (e == hipSuccess)
    e = launch_trmv_interp(p->d, k, M, q, c, L.ldz, th_t, wts, Z, a1, stream);
  if (e == hipSuccess)
    e = launch_trmv_interp(p->d, k, M, q, c, L.ldz, th_t, wts + 8 * q, Z, b1,
                           stream);
  if (e == hipSuccess)
    e = launch_trmv_interp(p->d, k, M, q, c, L.ldz, th_t, wts, Sg, a2, stream);
  if (e == hipSuccess)
    e = launch_trmv_interp(p->d, k, M, q, c, L.ldz, th_t, wts + 8 * q, Sg, b2,
                           stream);
  // <dLhat^T z, Lhat^T theta> + <Lhat^T z, dLhat^T theta>
  if (e == hipSuccess)
    e = launch_grad_dot(p->d, k, q, c, L.ldz, b2, a1, a2, b1, lamg, hn,
                        at<double>(ws, L.i_gpart), dlog, flags, stream);
  return hip_status(e);
}

pichol_status pichol_cv_exact_grad(const pichol_problem* p,
                                   const double* lam_grid, void* ws,
                                   size_t ws_bytes, double* err, double* dlog,
                                   double* W, int32_t* info, int32_t* flags,
                                   hipStream_t stream) {
  if (!problem_ok(p) || p->refine != 0 || !dlog) return PICHOL_ERR_ARG;
  const Layout L = layout_of(p);
  if (!ws || ws_bytes < L.e_gend) return PICHOL_ERR_WORKSPACE;
  pichol_status st =
      pichol_cv_exact(p, lam_grid, ws, ws_bytes, err, W, info, flags, stream);
  if (st != PICHOL_OK) return st;
  const int k = p->k, q = p->q, c = (int)p->c;
  double* Z = at<double>(ws, L.e_Z);
  double* Sg = at<double>(ws, L.e_gS);
  std::vector<double> zero(q, 0.0);
  HoldoutNorm hn;
  holdout_norm(p, &hn);
  hipError_t e =
      launch_store_doubles(zero.data(), q, at<double>(ws, L.e_gzero), stream);
  if (e == hipSuccess)
    e = launch_residual(p->d, k, q, c, L.ldz, at<double>(ws, L.G),
                        at<double>(ws, L.C), at<double>(ws, L.e_gzero), Z, Sg,
                        stream);
  if (e == hipSuccess)
    e = launch_solve_factors(p->d, k, q, c, at<double>(ws, L.e_L), L.ldz, Sg,
                             flags, at<double>(ws, L.e_linv),
                             at<double>(ws, L.e_X), stream);
  // dA/dlambda = I: <z, theta>
  if (e == hipSuccess)
    e = launch_grad_dot(p->d, k, q, c, L.ldz, Sg, Z, nullptr, nullptr,
                        at<double>(ws, L.e_lam), hn, at<double>(ws, L.e_gpart),
                        dlog, flags, stream);
  return hip_status(e);
}

pichol_status pichol_cv_pinrmse(const pichol_problem* p, const double* lam_s,
                                const double* lam_grid, double lam_ref,
                                void* ws, size_t ws_bytes, double* err,
                                double* err_s, int32_t* info, int32_t* flags,
                                hipStream_t stream) {
  if (!problem_ok(p) || p->refine != 0 || !lam_s || !lam_grid || !err ||
      !info || !flags || !(lam_ref > 0.0) || !isfinite(lam_ref))
    return PICHOL_ERR_ARG;
  if (!samples_ok(lam_s, p->g)) return PICHOL_ERR_ARG;
  for (int t = 0; t < p->q; ++t)
    if (!isfinite(lam_grid[t])) return PICHOL_ERR_ARG;
  if (!ws || ws_bytes < pinrmse_end(p)) return PICHOL_ERR_WORKSPACE;
  FitCoef fc;
  if (!basis_ok(p->basis, lam_s, p->g) || !basis_ok(p->basis, lam_grid, p->q))
    return PICHOL_ERR_ARG;
  if (!fit_coef(p->g, p->r, lam_s, lam_ref, p->basis, &fc)) return PICHOL_ERR_ARG;
  // exact hold-out errors at the g samples (the Gram blocks are shared)
  pichol_problem ps = *p;
  ps.q = p->g;
  double* es = err_s ? err_s : at<double>(ws, pinrmse_es(p));
  pichol_status st = pichol_cv_exact(&ps, lam_s, ws, ws_bytes, es, nullptr,
                                     info, flags, stream);
  if (st != PICHOL_OK) return st;
  double* tau = at<double>(ws, pinrmse_tau(p));
  hipError_t e = upload_tau(lam_grid, p->q, lam_ref, p->basis, tau, stream);
  if (e == hipSuccess) e = launch_pinrmse(p->k, fc, p->q, tau, es, err, stream);
  return hip_status(e);
}

int64_t pichol_vector_length(int64_t d, int32_t layout) {
  if (d < 1) return 0;
  int64_t n;
  if (layout == PICHOL_LAYOUT_ROWWISE || layout == PICHOL_LAYOUT_RECURSIVE)
    n = d * (d + 1) / 2;
  else if (layout == PICHOL_LAYOUT_FULL)
    n = d * d;
  else if (layout == PICHOL_LAYOUT_TILE)
    n = packed_elems_of(d);
  else
    return 0;
  return (n + 3) / 4 * 4;
}

pichol_status pichol_vectorize(int64_t d, int32_t nmat, const double* L,
                               int32_t layout, int32_t h0, double* T,
                               hipStream_t stream) {
  if (d < 1 || nmat < 1 || !L || !T || h0 < 1 ||
      (layout != PICHOL_LAYOUT_ROWWISE && layout != PICHOL_LAYOUT_FULL &&
       layout != PICHOL_LAYOUT_RECURSIVE))
    return PICHOL_ERR_ARG;
  const int kind = layout == PICHOL_LAYOUT_ROWWISE ? 1
                   : layout == PICHOL_LAYOUT_FULL  ? 2
                                                   : 3;
  return hip_status(launch_vectorize(d, nmat, L, kind, h0,
                                     pichol_vector_length(d, layout), T,
                                     stream));
}

pichol_status pichol_fit_vec(int64_t N, int32_t nmat, int32_t g, int32_t r,
                             const double* lam_s, double lam_ref,
                             const double* T, double* theta,
                             hipStream_t stream) {
  if (N < 4 || N % 4 || nmat < 1 || g < 1 || g > 32 || r < 0 || r > 7 ||
      r >= g || !lam_s || !T || !theta || !(lam_ref > 0.0) ||
      !isfinite(lam_ref))
    return PICHOL_ERR_ARG;
  if (!samples_ok(lam_s, g)) return PICHOL_ERR_ARG;
  FitCoef fc;
  if (!fit_coef(g, r, lam_s, lam_ref, 0, &fc)) return PICHOL_ERR_ARG;
  return hip_status(launch_fit_flat(N, nmat, fc, T, theta, stream));
}

pichol_status pichol_eval_vec(int64_t N, int32_t nmat, int32_t r,
                              const double* theta, int32_t nlam,
                              const double* lam, double lam_ref, double* out,
                              void* ws, size_t ws_bytes, hipStream_t stream) {
  if (N < 4 || N % 4 || nmat < 1 || r < 0 || r > 7 || nlam < 1 || !theta ||
      !lam || !out || !(lam_ref > 0.0) || !isfinite(lam_ref))
    return PICHOL_ERR_ARG;
  if (!ws || ws_bytes < pichol_lambda_workspace(nlam)) return PICHOL_ERR_WORKSPACE;
  double* tau = static_cast<double*>(ws);
  hipError_t e = upload_tau(lam, nlam, lam_ref, 0, tau, stream);
  if (e == hipSuccess)
    e = launch_eval_flat(N, nmat, r + 1, theta, nlam, tau, out, stream);
  return hip_status(e);
}

// The units of a pipeline call whose Gram-form hold-out error carries
// FLAG_CANCEL, recomputed from the residual R = Y_v - X_v W (slab Z).
static pichol_status holdout_direct_fix(const pichol_problem* p,
                                        const double* X, const double* Y,
                                        const double* Z, void* ws, double* err,
                                        int32_t* flags, hipStream_t stream) {
  const Layout L = layout_of(p);
  FoldSplit fs;
  fold_split(p->n, p->k, p->normalize, &fs);
  HoldoutNorm hn;
  holdout_norm(p, &hn);
  return hip_status(launch_holdout_direct(
      p->d, p->k, (int)p->c, p->q, L.ldz, Z, X, p->ldx, Y, p->ldy, fs, hn,
      at<double>(ws, L.dpart), err, flags, 1, stream));
}

pichol_status pichol_cv(const pichol_problem* p, const double* X,
                        const double* Y, const double* lam_s,
                        const double* lam_grid, double lam_ref, void* ws,
                        size_t ws_bytes, double* err, double* W, int32_t* info,
                        int32_t* flags, hipStream_t stream) {
  pichol_status st = pichol_cv_gram(p, X, Y, ws, ws_bytes, stream);
  if (st != PICHOL_OK) return st;
  st = pichol_cv_interp(p, lam_s, lam_grid, lam_ref, ws, ws_bytes, err, W,
                        info, flags, stream);
  if (st != PICHOL_OK) return st;
  return holdout_direct_fix(p, X, Y, at<double>(ws, layout_of(p).i_Z), ws, err,
                            flags, stream);
}

pichol_status pichol_exact_cv(const pichol_problem* p, const double* X,
                              const double* Y, const double* lam_grid, void* ws,
                              size_t ws_bytes, double* err, double* W,
                              int32_t* info, int32_t* flags,
                              hipStream_t stream) {
  pichol_status st = pichol_cv_gram(p, X, Y, ws, ws_bytes, stream);
  if (st != PICHOL_OK) return st;
  st = pichol_cv_exact(p, lam_grid, ws, ws_bytes, err, W, info, flags, stream);
  if (st != PICHOL_OK) return st;
  return holdout_direct_fix(p, X, Y, at<double>(ws, layout_of(p).e_Z), ws, err,
                            flags, stream);
}

pichol_status pichol_check(const int32_t* info, int64_t n_info,
                           const int32_t* flags, int64_t n_flags,
                           hipStream_t stream) {
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_status(e);
  std::vector<int32_t> h;
  if (info && n_info > 0) {
    h.resize(n_info);
    e = hipMemcpy(h.data(), info, sizeof(int32_t) * n_info, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_status(e);
    for (int32_t v : h)
      if (v != 0) return PICHOL_ERR_NOT_PD;
  }
  if (flags && n_flags > 0) {
    h.resize(n_flags);
    e = hipMemcpy(h.data(), flags, sizeof(int32_t) * n_flags, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_status(e);
    // bit2 (the Gram-form hold-out error is cancellation-limited) is
    // advisory; bits 0 and 1 are data errors
    for (int64_t i = 0; i < n_flags; ++i)
      if (h[i] & 3) return PICHOL_ERR_DATA;
  }
  return PICHOL_OK;
}

}  // extern "C"
