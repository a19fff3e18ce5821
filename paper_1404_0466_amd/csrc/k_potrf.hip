// Batched Cholesky factorization of shifted matrices H + lambda I
// (Sec. 3.2; Algorithm 1 step 1 and the exact per-lambda baseline).
//
// Blocked right-looking algorithm on 128-wide panels over the tile-packed
// layout.  For panel kk of every matrix in the batch:
//   1. k_potrf_diag   factors the diagonal tile in LDS and writes the
//                     inverse of the factor to a scratch tile;
//   2. k_potrf_panel  forms the tiles below it as A_{I,kk} L_kk^{-T}
//                     (an FP64 MFMA product with the inverse);
//   3. k_potrf_update subtracts L_{I,kk} L_{J,kk}^T from every trailing tile
//                     (FP64 MFMA, the bulk of the flops).
// One launch of each kernel covers the whole batch, so a batch of B
// matrices of order d fills the GPU with B * (trailing tiles) workgroups.
#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

// L(m*nshift + s) = H(m) + lam_s I: lower part copied, shift on the first d
// diagonal entries, identity padding, zeros above the diagonal of diagonal
// tiles.  Also clears info.
__global__ void __launch_bounds__(256) k_shift_copy(int64_t d, int64_t S,
                                                    const double* H,
                                                    int nshift,
                                                    const double* lam,
                                                    double* L, int* info) {
  const int64_t ms = blockIdx.y;
  const int64_t m = ms / nshift;
  const int s = (int)(ms % nshift);
  const int I = tri_row(blockIdx.x), J = blockIdx.x - (int)tri(I);
  const double shift = lam[s];
  const double* h = H + m * S + tile_off(I, J);
  double* l = L + ms * S + tile_off(I, J);
  for (int e = threadIdx.x; e < NB2; e += blockDim.x) {
    const int64_t i = (int64_t)I * NB + (e & (NB - 1));
    const int64_t j = (int64_t)J * NB + (e >> 7);
    double v;
    if (i >= d || j >= d)
      v = (i == j) ? 1.0 : 0.0;
    else if (i < j)
      v = 0.0;
    else
      v = h[e] + (i == j ? shift : 0.0);
    l[e] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) info[ms] = 0;
}

// Diagonal tile kk of factor f: unblocked right-looking Cholesky in LDS,
// then the in-place inverse of the factor.  Writes the factor tile and the
// inverse (column-major, zeros above the diagonal) to linv.
__global__ void __launch_bounds__(256) k_potrf_diag(int64_t d, int64_t S,
                                                    int kk, double* L,
                                                    int* info, double* linv) {
  __shared__ double a[NB * LDS_LD];
  __shared__ double tmp[NB];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  double* tile = L + (int64_t)f * S + tile_off(kk, kk);
  for (int e = tid; e < NB2; e += blockDim.x)
    a[(e >> 7) * LDS_LD + (e & (NB - 1))] = tile[e];
  __syncthreads();

  const int i = tid & (NB - 1), grp = tid >> 7;
  for (int j = 0; j < NB; ++j) {
    const double piv = a[j * LDS_LD + j];
    if (tid == 0 && !(piv > 0.0) && info[f] == 0 &&
        (int64_t)kk * NB + j < d)
      info[f] = kk * NB + j + 1;
    const double ljj = sqrt(piv);
    __syncthreads();  // every thread has read the pivot
    if (tid < NB) {
      if (i > j) a[j * LDS_LD + i] = a[j * LDS_LD + i] / ljj;
      if (i == j) a[j * LDS_LD + j] = ljj;
    }
    __syncthreads();
    if (i > j) {
      const double lij = a[j * LDS_LD + i];
      for (int c = j + 1 + grp; c <= i; c += 2)
        a[c * LDS_LD + i] -= lij * a[j * LDS_LD + c];
    }
    __syncthreads();
  }

  for (int e = tid; e < NB2; e += blockDim.x) {
    const int r = e & (NB - 1), c = e >> 7;
    tile[e] = (r >= c) ? a[c * LDS_LD + r] : 0.0;
  }
  __syncthreads();

  // In-place inverse, columns from last to first: with the trailing block
  // already inverted, column j becomes -(1/L_jj) * Tinv * x.
  for (int j = NB - 1; j >= 0; --j) {
    if (tid > j && tid < NB) tmp[tid] = a[j * LDS_LD + tid];
    __syncthreads();
    const double inv = 1.0 / a[j * LDS_LD + j];
    if (tid > j && tid < NB) {
      double y = 0.0;
      for (int p = j + 1; p <= tid; ++p) y += a[p * LDS_LD + tid] * tmp[p];
      a[j * LDS_LD + tid] = -inv * y;
    }
    __syncthreads();
    if (tid == j) a[j * LDS_LD + j] = inv;
  }
  __syncthreads();
  double* li = linv + (int64_t)f * NB2;
  for (int e = tid; e < NB2; e += blockDim.x) {
    const int r = e & (NB - 1), c = e >> 7;
    li[e] = (r >= c) ? a[c * LDS_LD + r] : 0.0;
  }
}

// Panel tile (I, kk), I > kk: X = A L_kk^{-T}, in place.  The wave computes
// D'(n,m) = sum_p Linv(n,p) A(m,p) = X(m,n), stored at n*128 + m.  Linv is
// lower triangular, so the sum stops at the wave's last n.
__global__ void __launch_bounds__(256) k_potrf_panel(int64_t S, int kk,
                                                     double* L,
                                                     const double* linv) {
  const int f = blockIdx.y;
  const int I = kk + 1 + blockIdx.x;
  const int w = threadIdx.x >> 6, wi = w >> 1, wj = w & 1;
  double* tile = L + (int64_t)f * S + tile_off(I, kk);
  const double* li = linv + (int64_t)f * NB2;
  Acc64 acc;
  acc.zero();
  mma_panel(acc, li + wi * 64, NB, tile + wj * 64, NB, wi * 64 + 64);
  __syncthreads();  // the whole tile is read before any part is overwritten
  const LaneXY lx;
  const int m0 = wj * 64 + lx.col0();
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const int n = wi * 64 + lx.row(v, bi);
      st4(tile + n * NB + m0, acc.row(v, bi));
    }
}

// Trailing tile (I,J), kk < J <= I: A_IJ -= sum_{c in [c0,c1)} L_Ic L_Jc^T.
// The wave computes D'(n,m) = sum_p L_Jc(n,p) L_Ic(m,p) = update(m,n).
__global__ void __launch_bounds__(256) k_potrf_update(int64_t S, int kk,
                                                      int c0, int c1,
                                                      double* L) {
  const int f = blockIdx.y;
  const int t = blockIdx.x;
  const int r = tri_row(t);
  const int I = kk + 1 + r, J = kk + 1 + (t - (int)tri(r));
  const int w = threadIdx.x >> 6, wi = w >> 1, wj = w & 1;
  if (I == J && wi > wj) return;  // block strictly above the diagonal
  double* Lf = L + (int64_t)f * S;
  Acc64 acc;
  acc.zero();
  for (int c = c0; c < c1; ++c)
    mma_panel(acc, Lf + tile_off(J, c) + wi * 64, NB,
              Lf + tile_off(I, c) + wj * 64, NB, NB);
  double* ct = Lf + tile_off(I, J);
  const LaneXY lx;
  const int m0 = wj * 64 + lx.col0();
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const int n = wi * 64 + lx.row(v, bi);
      double* p = ct + n * NB + m0;
      const v4d upd = acc.row(v, bi);
      if (I != J || wi != wj) {
        st4(p, ld4(p) - upd);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (m0 + e >= n) p[e] -= upd[e];
      }
    }
}

hipError_t launch_shift_copy(int64_t d, int nmat, const double* H, int nshift,
                             const double* lam_dev, double* L, int* info,
                             hipStream_t s) {
  const int64_t nt = ntiles_of(d);
  PICHOL_LAUNCH(k_shift_copy,
                     dim3((unsigned)tri(nt), (unsigned)(nmat * nshift)),
                     dim3(256), 0, s, d, packed_elems_of(d), H, nshift,
                     lam_dev, L, info);
  return hipGetLastError();
}

hipError_t launch_potrf_blocked(int64_t d, int nfac, double* L, int* info,
                                double* linv_ws, hipStream_t s) {
  const int nt = (int)ntiles_of(d);
  const int64_t S = packed_elems_of(d);
  for (int kk = 0; kk < nt; ++kk) {
    PICHOL_LAUNCH(k_potrf_diag, dim3((unsigned)nfac), dim3(256), 0, s, d,
                       S, kk, L, info, linv_ws);
    const int rest = nt - kk - 1;
    if (rest > 0) {
      PICHOL_LAUNCH(k_potrf_panel, dim3((unsigned)rest, (unsigned)nfac),
                         dim3(256), 0, s, S, kk, L, linv_ws);
      PICHOL_LAUNCH(k_potrf_update,
                         dim3((unsigned)tri(rest), (unsigned)nfac), dim3(256),
                         0, s, S, kk, kk, kk + 1, L);
    }
  }
  return hipGetLastError();
}

}  // namespace pichol
