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
    const double e = (yy[m] + s) / hn.count[m];
    err[m * q + t] = e;
    if (!isfinite(e)) flags[m * q + t] |= 1;
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

}  // namespace pichol
