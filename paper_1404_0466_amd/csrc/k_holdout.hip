// Hold-out error of every (fold, lambda).  With R = Y_v - X_v W the sum of
// squares is expanded as
//     |R|^2 = |Y_v|^2 - 2 <W, X_v^T Y_v> + <W, (X_v^T X_v) W>,
// using the validation block's Gram matrices from the Gram step, so the
// q*c solutions of a fold cost one FP64 MFMA product with the d x d block
// Gram instead of one with the n_v x d block of X.
// Reductions run in a fixed order (no floating-point atomics).
#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

// Partial sums over the rows of tile row I of
//     W(r, col) * ((G W)_h(r, col) - [h == 0] 2 C(r, col mod c))
// for the 128 slab columns of block cb, where (G W)_h sums over the column
// blocks J <= I of the h-th of HOLDOUT_KSPLIT ranges, the blocks J < I
// counted twice: G is symmetric, so <W, G W> = sum_I W_I^T (G_II W_I +
// 2 sum_{J<I} G_IJ W_J), half the products of the full sum (the expansion
// is linear in G W).  Written to partial[m][I][h][col]; a range that starts
// past I writes zeros.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_holdout_partial(
    int64_t d, int q, int c, int64_t ldz, const double* Z, const double* G,
    const double* C, double* partial) {
  __shared__ double red[64 * 2];
  const int cb = blockIdx.x;
  const int I = blockIdx.y;
  const int64_t m = blockIdx.z / HOLDOUT_KSPLIT;
  const int h = blockIdx.z % HOLDOUT_KSPLIT;
  const int w = threadIdx.x >> 6, wi = w >> 1, wj = w & 1;
  const int64_t nt = ntiles_of(d), dp = nt * NB;
  const int J0 = (int)(nt * h / HOLDOUT_KSPLIT);
  const int J1 = (int)(nt * (h + 1) / HOLDOUT_KSPLIT);
  const LaneXY lx;
  const int64_t col = (int64_t)cb * NB + wj * 64 + lx.col0();
  const int64_t qc = (int64_t)q * c;
  if (J0 > I) {  // the whole range lies above the diagonal
    if (wi == 0 && lx.lq == 0) {
      double* out = partial + ((m * nt + I) * HOLDOUT_KSPLIT + h) * ldz + col;
#pragma unroll
      for (int e = 0; e < 4; ++e) out[e] = 0.0;
    }
    return;
  }
  const double* gm = G + m * dp * dp + (int64_t)I * nt * NB2 + wi * 64;
  const double* zm = Z + m * dp * ldz + (int64_t)cb * NB + wj * 64;
  Acc64 acc;
  acc.zero();
  const int Jl = J1 < I ? J1 : I;  // blocks strictly below the diagonal
  for (int J = J0; J < Jl; ++J)
    mma_panel(acc, gm + (int64_t)J * NB2, NB, zm + (int64_t)J * NB * ldz, ldz,
              NB);
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc.c[bi][bj] *= 2.0;
  if (I < J1)
    mma_panel(acc, gm + (int64_t)I * NB2, NB, zm + (int64_t)I * NB * ldz, ldz,
              NB);
  const double c2 = h == 0 ? 2.0 : 0.0;

  int cmod[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) cmod[e] = (int)((col + e) % c);
  v4d part = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const int64_t r = (int64_t)I * NB + wi * 64 + lx.row(v, bi);
      const v4d wv = ld4(Z + (m * dp + r) * ldz + col);
      const v4d gw = acc.row(v, bi);
      const double* cr = C + (m * dp + r) * c;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        part[e] += wv[e] * (gw[e] - c2 * cr[cmod[e]]);
    }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double x = part[e];
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    part[e] = x;
  }
  // combine the two waves that share these columns
  if (wi == 1 && lx.lq == 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) red[wj * 64 + lx.col0() + e] = part[e];
  }
  __syncthreads();
  if (wi == 0 && lx.lq == 0) {
    double* out = partial + ((m * nt + I) * HOLDOUT_KSPLIT + h) * ldz + col;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double v = (col + e) < qc ? part[e] + red[wj * 64 + lx.col0() + e] : 0.0;
      out[e] = v;
    }
  }
}

// err[m][t] = (yy[m] + sum_I sum_j partial[m][I][t*c + j]) / (n_v * c).
__global__ void __launch_bounds__(64) k_holdout_final(int64_t nt, int q, int c,
                                                      int64_t ldz,
                                                      const double* partial,
                                                      const double* yy,
                                                      HoldoutNorm hn,
                                                      double* err, int* flags) {
  // one wavefront per (lambda t, fold m): lane l sums the partial rows
  // l, l + 64, ... in order, then a fixed butterfly adds the 64 lanes
  const int t = blockIdx.x;
  const int64_t m = blockIdx.y;
  const int l = threadIdx.x;
  const int64_t nI = nt * HOLDOUT_KSPLIT;
  double s = 0.0;
  for (int64_t I = l; I < nI; I += 64) {
    const double* p = partial + (m * nI + I) * ldz + (int64_t)t * c;
    for (int j = 0; j < c; ++j) s += p[j];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (l == 0) {
    const double sse = yy[m] + s;
    const double e = sse / hn.count[m];
    err[m * q + t] = e;
    int f = 0;
    if (!isfinite(e)) {
      f = 1;
    } else {
      // The expansion subtracts terms of the size of |Y_v|^2; its rounding
      // (G_v, C_v and the products: sums of about n_v and d terms) is
      // estimated as 4 eps |Y_v|^2 (sqrt(n_v) + sqrt(dp)).  Where that is
      // not below 1e-11 of the result, the unit is marked for the direct
      // residual (k_holdout_direct).
      const double nv = hn.count[m] / (double)c;
      const double est = yy[m] * (sqrt(nv) + sqrt((double)(nt * NB))) *
                         (4.0 * 0x1p-53);
      if (!(est <= 1e-11 * sse)) f = FLAG_CANCEL;
    }
    if (f) flags[m * q + t] |= f;
  }
}

hipError_t launch_holdout_partial(int64_t d, int nmat, int c, int q,
                                  int64_t ldz, const double* Z,
                                  const double* G, const double* C,
                                  double* partial, hipStream_t s) {
  const int64_t nt = ntiles_of(d);
  PICHOL_LAUNCH(k_holdout_partial,
                     dim3((unsigned)(ldz / NB), (unsigned)nt,
                          (unsigned)(nmat * HOLDOUT_KSPLIT)),
                     dim3(256), 0, s, d, q, c, ldz, Z, G, C, partial);
  return hipGetLastError();
}

hipError_t launch_holdout_final(int64_t d, int nmat, int c, int q, int64_t ldz,
                                const double* partial, const double* yy,
                                const HoldoutNorm& hn, double* err, int* flags,
                                hipStream_t s) {
  const int64_t nt = ntiles_of(d);
  PICHOL_LAUNCH(k_holdout_final, dim3((unsigned)q, (unsigned)nmat), dim3(64),
                     0, s, nt, q, c, ldz, partial, yy, hn, err, flags);
  return hipGetLastError();
}

hipError_t launch_holdout(int64_t d, int nmat, int c, int q, int64_t ldz,
                          const double* Z, const double* G, const double* C,
                          const double* yy, const HoldoutNorm& hn,
                          double* partial, double* err, int* flags,
                          hipStream_t s) {
  hipError_t e = launch_holdout_partial(d, nmat, c, q, ldz, Z, G, C, partial, s);
  if (e != hipSuccess) return e;
  return launch_holdout_final(d, nmat, c, q, ldz, partial, yy, hn, err, flags,
                              s);
}

// ---------------------------------------------------------------------------
// Direct hold-out residual: the definition R = Y_v - X_v W, for the units
// where the Gram expansion above cancels (a well-fitted target, |R|^2 much
// smaller than |Y_v|^2) or, from pichol_holdout_direct, for every unit.
//
// The product X_v W runs on FP64 MFMA with no LDS.  The wave block is
//     D'(i, j) = sum_k Z(k, c0 + i) X(v0 + j0 + j, k)
// (i: slab column, j: validation row).  Z is read along its rows as in
// mma_panel.  X is row-major, contiguous in k, so a lane loads four
// consecutive k of one row with one 32-byte load and spends them in four
// consecutive MFMA steps: in step s of a 16-wide k chunk, lane group
// lq = l/16 carries k = k0 + 4 lq + s on both operands, the same
// permutation of the chunk's k order on either side.
// ---------------------------------------------------------------------------

__device__ inline v4d ld4_row_masked(const double* rowp, int64_t k, int64_t d) {
  v4d v = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (k + e < d) v[e] = rowp[k + e];
  return v;
}

// Partial sums sum_j R(j, col)^2 over the 128 validation rows of row block
// rb of fold m, for the 128 slab columns of block cb, written to
// partial[m][rb][col].  With only_flagged, a workgroup whose columns meet no
// lambda marked FLAG_CANCEL returns at once (its partial sums are never
// read).
__global__ void __launch_bounds__(256) k_holdout_direct(
    int64_t d, int q, int c, int64_t ldz, const double* Z, const double* X,
    int64_t ldx, const double* Y, int64_t ldy, FoldSplit fs, const int* flags,
    int only_flagged, int vec_ok, int64_t nrb, double* partial) {
  __shared__ double red[2][2][64];
  const int cb = blockIdx.x, rb = blockIdx.y, m = blockIdx.z;
  const int64_t v0 = fs.start[m], nv = fs.start[m + 1] - v0;
  const int64_t j0 = (int64_t)rb * NB;
  const int64_t qc = (int64_t)q * c, c0 = (int64_t)cb * NB;
  if (j0 >= nv || c0 >= qc) return;
  if (only_flagged) {
    const int64_t t0 = c0 / c;
    int64_t t1 = (c0 + NB - 1) / c;
    if (t1 > q - 1) t1 = q - 1;
    bool any = false;
    for (int64_t t = t0; t <= t1; ++t)
      any = any || (flags[(int64_t)m * q + t] & FLAG_CANCEL) != 0;
    if (!any) return;
  }
  const int w = threadIdx.x >> 6, wi = w >> 1, wj = w & 1;
  const LaneXY lx;
  const int64_t dp = ntiles_of(d) * NB;
  const double* zb = Z + (int64_t)m * dp * ldz + c0 + wi * 64 + 4 * lx.lr;
  // the lane's validation rows j = 4 lr + bj of the wave's 64 (rows past the
  // fold read row 0 and are zeroed)
  const double* xr[4];
  bool rok[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    const int64_t j = j0 + wj * 64 + 4 * lx.lr + bj;
    rok[bj] = j < nv;
    xr[bj] = X + (v0 + (rok[bj] ? j : 0)) * ldx;
  }
  const v4d zero = {0.0, 0.0, 0.0, 0.0};
  const int64_t kend = (d + 15) / 16 * 16;  // <= dp; slab rows >= d are 0
  Acc64 acc;
  acc.zero();
  v4d av[4], bv[4];
  auto load = [&](int64_t k0) {
    const int64_t kk = k0 + 4 * lx.lq;
#pragma unroll
    for (int s = 0; s < 4; ++s) av[s] = ld4(zb + (kk + s) * ldz);
    const bool full = vec_ok && k0 + 16 <= d;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const v4d x = full ? ld4(xr[bj] + kk) : ld4_row_masked(xr[bj], kk, d);
      bv[bj] = rok[bj] ? x : zero;
    }
  };
  load(0);
  for (int64_t k0 = 0; k0 < kend; k0 += 16) {
    v4d a[4], b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a[s] = av[s];
      b[s] = bv[s];
    }
    if (k0 + 16 < kend) load(k0 + 16);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
          acc.c[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              a[s][bi], b[bj][s], acc.c[bi][bj], 0, 0, 0);
  }
  // element v of block (bi, bj): D'(16v + 4lq + bi, 4lr + bj)
  double cs[4][4];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const int64_t col = c0 + wi * 64 + lx.row(v, bi);
      const bool cok = col < qc;
      const int64_t yc = cok ? col % c : 0;
      double s = 0.0;
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) {
        const int64_t j = j0 + wj * 64 + 4 * lx.lr + bj;
        const bool ok = cok && rok[bj];
        const double y = ok ? Y[(v0 + j) * ldy + yc] : 0.0;
        const double r = ok ? y - acc.c[bi][bj][v] : 0.0;
        s += r * r;
      }
      // the 16 lanes of this lane group hold the other rows
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      s += __shfl_xor(s, 4);
      s += __shfl_xor(s, 8);
      cs[v][bi] = s;
    }
  if (lx.lr == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) red[wi][wj][lx.row(v, bi)] = cs[v][bi];
  }
  __syncthreads();
  if (threadIdx.x < 128) {
    const int h = threadIdx.x >> 6, i = threadIdx.x & 63;
    partial[((int64_t)m * nrb + rb) * ldz + c0 + h * 64 + i] =
        red[h][0][i] + red[h][1][i];
  }
}

// err[m][t] = sum_rb sum_j partial[m][rb][t*c + j] / (n_v * c) for the units
// marked FLAG_CANCEL (or every unit), whose flag bit is then cleared.
__global__ void __launch_bounds__(64) k_holdout_direct_final(
    int q, int c, int64_t ldz, int64_t nrb, FoldSplit fs, const double* partial,
    HoldoutNorm hn, double* err, int* flags, int only_flagged) {
  const int t = blockIdx.x;
  const int64_t m = blockIdx.y;
  const int l = threadIdx.x;
  int* fl = flags + m * q + t;
  const int f0 = *fl;
  if (only_flagged && !(f0 & FLAG_CANCEL)) return;
  const int64_t nv = fs.start[m + 1] - fs.start[m];
  const int64_t nr = (nv + NB - 1) / NB;
  double s = 0.0;
  for (int64_t rb = l; rb < nr; rb += 64) {
    const double* p = partial + (m * nrb + rb) * ldz + (int64_t)t * c;
    for (int j = 0; j < c; ++j) s += p[j];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (l == 0) {
    const double e = s / hn.count[m];
    err[m * q + t] = e;
    int f = f0 & ~FLAG_CANCEL;
    if (!isfinite(e)) f |= 1;
    *fl = f;
  }
}

int64_t holdout_direct_rowblocks(const FoldSplit& fs) {
  int64_t mx = 0;
  for (int f = 0; f < fs.k; ++f) {
    const int64_t nv = fs.start[f + 1] - fs.start[f];
    if (nv > mx) mx = nv;
  }
  return (mx + NB - 1) / NB;
}

hipError_t launch_holdout_direct(int64_t d, int nmat, int c, int q,
                                 int64_t ldz, const double* Z, const double* X,
                                 int64_t ldx, const double* Y, int64_t ldy,
                                 const FoldSplit& fs, const HoldoutNorm& hn,
                                 double* partial, double* err, int* flags,
                                 int only_flagged, hipStream_t s) {
  const int64_t nrb = holdout_direct_rowblocks(fs);
  const int vec_ok = ((ldx & 3) == 0) && ((((uintptr_t)X) & 31) == 0);
  PICHOL_LAUNCH(k_holdout_direct,
                dim3((unsigned)(ldz / NB), (unsigned)nrb, (unsigned)nmat),
                dim3(256), 0, s, d, q, c, ldz, Z, X, ldx, Y, ldy, fs, flags,
                only_flagged, vec_ok, nrb, partial);
  PICHOL_LAUNCH(k_holdout_direct_final, dim3((unsigned)q, (unsigned)nmat),
                dim3(64), 0, s, q, c, ldz, nrb, fs, partial, hn, err, flags,
                only_flagged);
  return hipGetLastError();
}

}  // namespace pichol
