// Batched cross-validation of many independent ridge problems
// (pichol_cv_batch and its HIP-graph form).
//
// Problems that share their shape (d, c, k, g, r, q, precision) and, for the
// interpolated method, their scaled sample and grid values form a bucket.
// The stacked matrices of a bucket (problems x folds) are one batch for
// every kernel after the Gram step, so a bucket of B problems costs the
// launches of one problem with B*k folds; each problem keeps its own shifts,
// fold split and hold-out counts.  Buckets are independent: they are spread
// over up to four library-owned streams, forked from and joined back to the
// caller's stream with events, which also makes the whole call capturable.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "api_internal.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "pichol.h"

struct pichol_graph_s {
  hipGraphExec_t exec;
};

namespace pichol {
namespace {

constexpr int kMaxStreams = 4;

struct Bucket {
  std::vector<int> items;  // indices into the batch, in input order
  int64_t d = 0, c = 0;
  int k = 0, g = 0, r = 0, q = 0, precision = 0;
  double cost = 0.0;       // estimated work, for the stream assignment
  int64_t nrb = 0;         // row blocks of the largest validation fold
  int stream = 0;
  size_t base = 0;         // byte offset of the bucket's workspace region
  // region offsets, relative to base
  size_t G, C, yy, H, Bm, lam, tau, L, linv, th, tht, Z, X, part, dinv,
      dpart, info, flags, end;
};

// Scaled values lambda/lam_ref of two problems agree to a few ulps (they are
// computed from differently scaled lambdas, so exact equality is too
// strict); the bucket then uses its first problem's values.
bool close_ratio(double x, double y) {
  const double m = fabs(x) > fabs(y) ? fabs(x) : fabs(y);
  return fabs(x - y) <= 8.0 * 2.220446049250313e-16 * m;
}

bool same_bucket(const pichol_batch_item& a, const pichol_batch_item& b,
                 int method) {
  const pichol_problem &p = a.p, &o = b.p;
  if (p.d != o.d || p.c != o.c || p.k != o.k || p.q != o.q ||
      p.precision != o.precision || p.basis != o.basis)
    return false;
  if (method != PICHOL_METHOD_INTERP) return true;
  if (p.g != o.g || p.r != o.r) return false;
  for (int s = 0; s < p.g; ++s)
    if (!close_ratio(a.lam_s[s] / a.lam_ref, b.lam_s[s] / b.lam_ref))
      return false;
  for (int t = 0; t < p.q; ++t)
    if (!close_ratio(a.lam_grid[t] / a.lam_ref, b.lam_grid[t] / b.lam_ref))
      return false;
  return true;
}

bool item_ok(const pichol_batch_item& it, int method) {
  const pichol_problem& p = it.p;
  if (!problem_ok(&p) || p.refine != 0) return false;
  if (!it.X || !it.Y || !it.lam_grid || !it.err || !it.info || !it.flags)
    return false;
  for (int t = 0; t < p.q; ++t)
    if (!isfinite(it.lam_grid[t])) return false;
  if (method == PICHOL_METHOD_INTERP) {
    if (!it.lam_s || !(it.lam_ref > 0.0) || !isfinite(it.lam_ref)) return false;
    if (!samples_ok(it.lam_s, p.g)) return false;
    if (!basis_ok(p.basis, it.lam_s, p.g) || !basis_ok(p.basis, it.lam_grid, p.q))
      return false;
    FitCoef fc;
    if (!fit_coef(p.g, p.r, it.lam_s, it.lam_ref, p.basis, &fc)) return false;
  }
  return true;
}

void layout_bucket(Bucket& b, int method) {
  const size_t dbl = sizeof(double), i32 = sizeof(int32_t);
  const int64_t nt = ntiles_of(b.d), dp = nt * NB;
  const int64_t S = packed_elems_of(b.d);
  const int64_t ldz = (int64_t)(b.q * b.c + NB - 1) / NB * NB;
  const size_t nb = b.items.size(), nmat = nb * (size_t)b.k;
  const size_t q = (size_t)b.q, M = (size_t)b.r + 1;
  const size_t nf = method == PICHOL_METHOD_INTERP ? (size_t)b.g : q;
  size_t o = 0;
  b.G = o; o += align256(nmat * dp * dp * dbl);
  b.C = o; o += align256(nmat * dp * b.c * dbl);
  b.yy = o; o += align256(nmat * dbl);
  b.H = o; o += align256(nmat * S * dbl);
  b.Bm = o; o += align256(nmat * dp * b.c * dbl);
  b.lam = o; o += align256(nb * nf * dbl);
  b.tau = o; o += align256(q * dbl);
  b.L = o; o += align256(nmat * nf * S * dbl);
  // exact factors keep the inverse of every diagonal tile for the solves
  b.linv = o;
  o += align256(nmat * nf * (method == PICHOL_METHOD_INTERP ? 1 : nt) * NB2 * dbl);
  const bool interp = method == PICHOL_METHOD_INTERP;
  b.th = o; o += interp ? align256(nmat * M * S * dbl) : 0;
  b.tht = o; o += interp ? align256(nmat * M * S * dbl) : 0;
  b.Z = o; o += align256(nmat * dp * ldz * dbl);
  b.X = o; o += align256(nmat * dp * ldz * dbl);
  b.part = o; o += align256(nmat * nt * HOLDOUT_KSPLIT * ldz * dbl);
  b.dinv = o; o += interp ? align256(nmat * q * nt * NB2 * dbl) : 0;
  // direct hold-out partial sums, shared by the bucket's problems in turn
  b.dpart = o; o += align256((size_t)b.k * b.nrb * ldz * dbl);
  b.info = o; o += align256(nmat * nf * i32);
  b.flags = o; o += align256(nmat * q * i32);
  b.end = o;
}

// Group the items into buckets (first-appearance order) and lay out their
// workspace regions one after another.  Returns false on an invalid item.
bool make_buckets(int nprob, const pichol_batch_item* items, int method,
                  std::vector<Bucket>* out, size_t* total) {
  if (nprob < 1 || !items ||
      (method != PICHOL_METHOD_INTERP && method != PICHOL_METHOD_EXACT))
    return false;
  std::vector<Bucket>& bs = *out;
  bs.clear();
  for (int i = 0; i < nprob; ++i) {
    if (!item_ok(items[i], method)) return false;
    Bucket* hit = nullptr;
    for (Bucket& b : bs)
      if (same_bucket(items[b.items[0]], items[i], method)) {
        hit = &b;
        break;
      }
    if (!hit) {
      bs.emplace_back();
      hit = &bs.back();
      const pichol_problem& p = items[i].p;
      hit->d = p.d;
      hit->c = p.c;
      hit->k = p.k;
      hit->g = p.g;
      hit->r = p.r;
      hit->q = p.q;
      hit->precision = p.precision;
    }
    hit->items.push_back(i);
    FoldSplit fs;
    fold_split(items[i].p.n, items[i].p.k, items[i].p.normalize, &fs);
    hit->nrb = std::max(hit->nrb, holdout_direct_rowblocks(fs));
  }
  size_t base = 0;
  for (Bucket& b : bs) {
    layout_bucket(b, method);
    b.base = base;
    base += b.end;
    const double d3 = (double)b.d * (double)b.d * (double)b.d;
    const double nfac = (double)b.items.size() * b.k *
                        (method == PICHOL_METHOD_INTERP ? b.g : b.q);
    b.cost = nfac * d3 / 3.0 +
             2.0 * (double)b.items.size() * b.k * (double)b.d * b.d * b.q * b.c;
  }
  *total = base;
  return true;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// One bucket's pipeline on stream st.
hipError_t run_bucket(const Bucket& b, const pichol_batch_item* items,
                      int method, int group, int form, void* ws, hipStream_t st) {
  const bool interp = method == PICHOL_METHOD_INTERP;
  const int64_t d = b.d, nt = ntiles_of(d), dp = nt * NB;
  const int64_t S = packed_elems_of(d);
  const int c = (int)b.c, k = b.k, q = b.q, M = b.r + 1;
  const int nf = interp ? b.g : q;
  const int64_t ldz = (int64_t)(q * c + NB - 1) / NB * NB;
  const int nb = (int)b.items.size(), nmat = nb * k;
  char* base = static_cast<char*>(ws) + b.base;
  double* G = at<double>(base, b.G);
  double* C = at<double>(base, b.C);
  double* yy = at<double>(base, b.yy);
  double* H = at<double>(base, b.H);
  double* Bm = at<double>(base, b.Bm);
  double* lam = at<double>(base, b.lam);
  double* tau = at<double>(base, b.tau);
  double* L = at<double>(base, b.L);
  double* linv = at<double>(base, b.linv);
  double* Z = at<double>(base, b.Z);
  double* part = at<double>(base, b.part);
  int* info = at<int>(base, b.info);
  int* flags = at<int>(base, b.flags);
  hipError_t e = hipSuccess;
  // fold Gram blocks of every problem into its slots of the stacked arrays
  std::vector<double> lam_all((size_t)nb * nf);
  for (int li = 0; li < nb && e == hipSuccess; ++li) {
    const pichol_batch_item& it = items[b.items[li]];
    FoldSplit fs;
    fold_split(it.p.n, k, it.p.normalize, &fs);
    const int64_t m0 = (int64_t)li * k;
    e = launch_gram(it.X, it.p.ldx, it.Y, it.p.ldy, d, c, fs, G + m0 * dp * dp,
                    C + m0 * dp * c, yy + m0, H + m0 * S, Bm + m0 * dp * c, st);
    const double* src = interp ? it.lam_s : it.lam_grid;
    for (int s = 0; s < nf; ++s) lam_all[(size_t)li * nf + s] = src[s];
  }
  if (e == hipSuccess) e = launch_store_doubles(lam_all.data(), nb * nf, lam, st);
  if (e == hipSuccess)
    e = launch_potrf_blocked(d, nmat * nf, ShiftSrc{H, nf, lam, k}, L, info,
                             linv, interp ? 0 : 1,
                             b.precision == PICHOL_PREC_MIXED, 0, group, st);
  if (e == hipSuccess)
    e = launch_slab_init(d, nmat, q, c, ldz, Bm, Z, flags, st);
  if (interp) {
    const pichol_batch_item& it0 = items[b.items[0]];
    FitCoef fc;
    fit_coef(b.g, b.r, it0.lam_s, it0.lam_ref, it0.p.basis, &fc);
    double* th = at<double>(base, b.th);
    double* tht = at<double>(base, b.tht);
    if (e == hipSuccess)
      e = upload_tau(it0.lam_grid, q, it0.lam_ref, it0.p.basis, tau, st);
    if (e == hipSuccess) e = launch_fit(d, nmat, fc, L, th, tht, st);
    if (e == hipSuccess)
      e = launch_solve_interp(d, nmat, c, M, th, tht, q, tau, ldz, Z,
                              at<double>(base, b.X), flags,
                              at<double>(base, b.dinv), 1, st, 0, form);
  } else {
    if (e == hipSuccess)
      e = launch_solve_factors(d, nmat, q, c, L, ldz, Z, flags, linv,
                               at<double>(base, b.X), st);
  }
  if (e == hipSuccess)
    e = launch_holdout_partial(d, nmat, c, q, ldz, Z, G, C, part, st);
  // per problem: hold-out errors straight into its err, status words and
  // weights gathered out of the stacked arrays
  for (int li = 0; li < nb && e == hipSuccess; ++li) {
    const pichol_batch_item& it = items[b.items[li]];
    const int64_t m0 = (int64_t)li * k;
    HoldoutNorm hn;
    holdout_norm(&it.p, &hn);
    e = launch_holdout_final(d, k, c, q, ldz,
                             part + m0 * nt * HOLDOUT_KSPLIT * ldz, yy + m0, hn,
                             it.err, flags + m0 * q, st);
    // units where the Gram form cancels: the residual from X and Y
    if (e == hipSuccess) {
      FoldSplit fs;
      fold_split(it.p.n, k, it.p.normalize, &fs);
      e = launch_holdout_direct(d, k, c, q, ldz, Z + m0 * dp * ldz, it.X,
                                it.p.ldx, it.Y, it.p.ldy, fs, hn,
                                at<double>(base, b.dpart), it.err,
                                flags + m0 * q, 1, st);
    }
    if (e == hipSuccess)
      e = launch_copy_i32((int64_t)k * nf, info + m0 * nf, it.info, st);
    if (e == hipSuccess)
      e = launch_copy_i32((int64_t)k * q, flags + m0 * q, it.flags, st);
    if (e == hipSuccess && it.W)
      e = launch_slab_to_weights(d, k, q, c, ldz, Z + m0 * dp * ldz, it.W, st);
  }
  return e;
}

// Library-owned streams for independent buckets, per device.
struct BatchStreams {
  bool ready = false;
  hipStream_t st[kMaxStreams];
  hipEvent_t fork;
  hipEvent_t join[kMaxStreams];
};
BatchStreams g_bs[64];
std::mutex g_bs_mu;

hipError_t batch_streams(BatchStreams** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  BatchStreams& bs = g_bs[dev];
  if (!bs.ready) {
    for (int i = 0; i < kMaxStreams && e == hipSuccess; ++i)
      e = hipStreamCreateWithFlags(&bs.st[i], hipStreamNonBlocking);
    if (e == hipSuccess)
      e = hipEventCreateWithFlags(&bs.fork, hipEventDisableTiming);
    for (int i = 0; i < kMaxStreams && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&bs.join[i], hipEventDisableTiming);
    if (e != hipSuccess) return e;
    bs.ready = true;
  }
  *out = &bs;
  return hipSuccess;
}

// Stream assignment: decreasing cost onto the least-loaded stream, or input
// order round-robin.
void assign_streams(std::vector<Bucket>& bs, int nstreams, int order,
                    std::vector<int>* run_order) {
  std::vector<int> idx(bs.size());
  for (size_t i = 0; i < bs.size(); ++i) idx[i] = (int)i;
  if (order == 0)
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int a, int b) { return bs[a].cost > bs[b].cost; });
  std::vector<double> load(nstreams, 0.0);
  for (size_t j = 0; j < idx.size(); ++j) {
    Bucket& b = bs[idx[j]];
    int s = (int)(j % nstreams);
    if (order == 0)
      s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b.stream = s;
    load[s] += b.cost;
  }
  *run_order = idx;
}

}  // namespace
}  // namespace pichol

using namespace pichol;

extern "C" {

pichol_status pichol_batch_workspace_size(int32_t nprob,
                                          const pichol_batch_item* items,
                                          int32_t method, size_t* bytes) {
  if (!bytes) return PICHOL_ERR_ARG;
  std::vector<Bucket> bs;
  size_t total = 0;
  if (!make_buckets(nprob, items, method, &bs, &total)) return PICHOL_ERR_ARG;
  *bytes = total;
  return PICHOL_OK;
}

int32_t pichol_batch_buckets(int32_t nprob, const pichol_batch_item* items,
                             int32_t method) {
  std::vector<Bucket> bs;
  size_t total = 0;
  if (!make_buckets(nprob, items, method, &bs, &total)) return -1;
  return (int32_t)bs.size();
}

pichol_status pichol_cv_batch(int32_t nprob, const pichol_batch_item* items,
                              int32_t method, const pichol_batch_tuning* tune,
                              void* ws, size_t ws_bytes, hipStream_t stream) {
  std::vector<Bucket> bs;
  size_t total = 0;
  if (!make_buckets(nprob, items, method, &bs, &total)) return PICHOL_ERR_ARG;
  int nstreams = kMaxStreams, order = 0;
  if (tune) {
    if (tune->streams < 0 || tune->streams > kMaxStreams || tune->order < 0 ||
        tune->order > 1)
      return PICHOL_ERR_ARG;
    for (int i = 0; i < 32; ++i)
      if (tune->panel_group[i] < 0 || tune->panel_group[i] > 8 ||
          tune->solve_form[i] < 0 || tune->solve_form[i] > 2)
        return PICHOL_ERR_ARG;
    if (tune->streams > 0) nstreams = tune->streams;
    order = tune->order;
  }
  // panels per delayed update for a bucket of nt tile rows (0: option)
  auto group_of = [&](const Bucket& b) {
    const int64_t nt = ntiles_of(b.d);
    return (tune && nt >= 1 && nt <= 32) ? tune->panel_group[nt - 1] : 0;
  };
  // form of the interpolated solves for the bucket (0: option / automatic)
  auto form_of = [&](const Bucket& b) {
    const int64_t nt = ntiles_of(b.d);
    return (tune && nt >= 1 && nt <= 32) ? tune->solve_form[nt - 1] : 0;
  };
  if (!ws || ws_bytes < total) return PICHOL_ERR_WORKSPACE;
  if (nstreams > (int)bs.size()) nstreams = (int)bs.size();
  std::vector<int> run_order;
  assign_streams(bs, nstreams, order, &run_order);
  if (nstreams == 1) {
    hipError_t e = hipSuccess;
    for (int j : run_order) {
      e = run_bucket(bs[j], items, method, group_of(bs[j]), form_of(bs[j]), ws,
                     stream);
      if (e != hipSuccess) break;
    }
    return hip_status(e);
  }
  std::lock_guard<std::mutex> lk(g_bs_mu);
  BatchStreams* S = nullptr;
  hipError_t e = batch_streams(&S);
  if (e != hipSuccess) return hip_status(e);
  e = hipEventRecord(S->fork, stream);
  for (int i = 0; i < nstreams && e == hipSuccess; ++i)
    e = hipStreamWaitEvent(S->st[i], S->fork, 0);
  for (int j : run_order) {
    if (e != hipSuccess) break;
    e = run_bucket(bs[j], items, method, group_of(bs[j]), form_of(bs[j]), ws,
                   S->st[bs[j].stream]);
  }
  // join every forked stream back, also after a failure, so that no stream
  // is left depending on work the caller does not wait for
  for (int i = 0; i < nstreams; ++i) {
    hipError_t e2 = hipEventRecord(S->join[i], S->st[i]);
    if (e2 == hipSuccess) e2 = hipStreamWaitEvent(stream, S->join[i], 0);
    if (e == hipSuccess) e = e2;
  }
  return hip_status(e);
}

pichol_status pichol_cv_batch_graph(int32_t nprob,
                                    const pichol_batch_item* items,
                                    int32_t method,
                                    const pichol_batch_tuning* tune, void* ws,
                                    size_t ws_bytes, pichol_graph* graph) {
  if (!graph || profiling_on()) return PICHOL_ERR_ARG;
  *graph = nullptr;
  std::vector<Bucket> bs;
  size_t total = 0;
  if (!make_buckets(nprob, items, method, &bs, &total)) return PICHOL_ERR_ARG;
  if (!ws || ws_bytes < total) return PICHOL_ERR_WORKSPACE;
  {
    // create the library streams before capturing
    std::lock_guard<std::mutex> lk(g_bs_mu);
    BatchStreams* S = nullptr;
    hipError_t e = batch_streams(&S);
    if (e != hipSuccess) return hip_status(e);
  }
  prepare_gram();
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_status(e);
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return hip_status(e);
  }
  pichol_status st = pichol_cv_batch(nprob, items, method, tune, ws, ws_bytes, cs);
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(cs, &g);
  hipGraphExec_t exec = nullptr;
  if (st == PICHOL_OK && ee == hipSuccess)
    ee = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (st != PICHOL_OK) return st;
  if (ee != hipSuccess) return hip_status(ee);
  pichol_graph out = new (std::nothrow) pichol_graph_s{exec};
  if (!out) {
    (void)hipGraphExecDestroy(exec);
    return PICHOL_ERR_ARG;
  }
  *graph = out;
  return PICHOL_OK;
}

pichol_status pichol_graph_begin(hipStream_t stream) {
  if (!stream || profiling_on() || option_lookahead()) return PICHOL_ERR_ARG;
  {
    // the batch streams must exist before any capture that may use them
    std::lock_guard<std::mutex> lk(g_bs_mu);
    BatchStreams* S = nullptr;
    hipError_t e = batch_streams(&S);
    if (e != hipSuccess) return hip_status(e);
  }
  prepare_gram();
  return hip_status(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
}

pichol_status pichol_graph_end(hipStream_t stream, pichol_graph* graph) {
  if (!stream || !graph) return PICHOL_ERR_ARG;
  *graph = nullptr;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(stream, &g);
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_status(e);
  pichol_graph out = new (std::nothrow) pichol_graph_s{exec};
  if (!out) {
    (void)hipGraphExecDestroy(exec);
    return PICHOL_ERR_ARG;
  }
  *graph = out;
  return PICHOL_OK;
}

pichol_status pichol_graph_launch(pichol_graph graph, hipStream_t stream) {
  if (!graph) return PICHOL_ERR_ARG;
  return hip_status(hipGraphLaunch(graph->exec, stream));
}

pichol_status pichol_graph_destroy(pichol_graph graph) {
  if (!graph) return PICHOL_ERR_ARG;
  hipError_t e = hipGraphExecDestroy(graph->exec);
  delete graph;
  return hip_status(e);
}

}  // extern "C"
