// Derivative of the hold-out error with respect to log lambda (the
// differentiation form of the method).
//
// With A = Lhat Lhat^T at lambda (Sec. 3.3's interpolated factor),
// theta = A^{-1} B_f, R = Y_v - X_v theta and z = A^{-1} X_v^T R:
//   d mse / d lambda = 2/(n_v c) <z, (dLhat Lhat^T + Lhat dLhat^T) theta>
//                    = 2/(n_v c) (<dLhat^T z, Lhat^T theta> + <Lhat^T z, dLhat^T theta>),
// dLhat = sum_j j tau^(j-1) / lambda_ref Theta_j.  X_v^T R = C_v - G_v theta
// comes from the validation block's Gram matrices (k_residual with a zero
// shift), z from one more pair of interpolated solves, and the four
// transposed products from k_trmv_interp: one FP64 MFMA product per tile
// row over the coefficient planes, with per-lambda column weights.  For
// exact factors dA/dlambda = I and the product is <z, theta>.
#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

// Out rows of tile I, slab columns of block cb:
//   Out_I = sum_{J >= I} sum_p Theta_p(J,I)^T (w_p(col) .* X_J),
// i.e. (sum_p w_p Theta_p)^T X per lambda, with w[p*q + t] the weight of
// plane p for lambda t (columns t*c .. t*c+c-1).  The transposed tiles are
// read from the row-major copy of the planes.  Four waves own 64 x 64
// quarters of the 128 x 128 output block.
__global__ void __launch_bounds__(256) k_trmv_interp(
    int64_t dp, int nt, const double* theta_t, int64_t S, int M, int q, int c,
    int64_t ldz, int ncb, const double* w, const double* X, double* Out) {
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int cb = id % ncb;
  const int rest = id / ncb;
  const int I = rest % nt;
  const int64_t m = rest / nt;
  const int wv = threadIdx.x >> 6, wi = wv >> 1, wj = wv & 1;
  const LaneXY lx;
  const int64_t col = (int64_t)cb * NB + wj * 64 + lx.col0();
  const int64_t qc = (int64_t)q * c;
  v4d wp[8];
#pragma unroll
  for (int p = 0; p < 8; ++p)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      wp[p][e] = (p < M && (col + e) < qc) ? w[p * q + (col + e) / c] : 0.0;
  Acc64 acc;
  acc.zero();
  const double* planes = theta_t + m * M * S;
  const double* xb = X + m * dp * ldz + (int64_t)cb * NB + wj * 64;
  for (int J = I; J < nt; ++J) {
    const double* tile = planes + tile_off(J, I) + wi * 64;
    const double* xj = xb + (int64_t)J * NB * ldz;
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (p < M) mma_panel_scaled(acc, tile + p * S, NB, xj, ldz, NB, wp[p]);
  }
  const int64_t row0 = m * dp + (int64_t)I * NB + wi * 64;
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
      st4(Out + (row0 + lx.row(v, bi)) * ldz + col, acc.row(v, bi));
}

// partial[(m*nt + I)*q + t] = sum over the rows of tile I and the c columns
// of lambda t of x1 .* y1 (+ x2 .* y2 when x2 is given), rows in increasing
// order then columns in increasing order.
__global__ void __launch_bounds__(256) k_grad_partial(
    int nt, int q, int c, int64_t ldz, const double* x1, const double* y1,
    const double* x2, const double* y2, double* partial) {
  const int I = blockIdx.x;
  const int64_t m = blockIdx.y;
  const int64_t dp = (int64_t)nt * NB;
  for (int t = threadIdx.x; t < q; t += blockDim.x) {
    double acc = 0.0;
    for (int r = 0; r < NB; ++r) {
      const int64_t o = (m * dp + (int64_t)I * NB + r) * ldz + (int64_t)t * c;
      for (int j = 0; j < c; ++j) {
        acc += x1[o + j] * y1[o + j];
        if (x2) acc += x2[o + j] * y2[o + j];
      }
    }
    partial[(m * nt + I) * q + t] = acc;
  }
}

// dlog[m*q + t] = lambda_t * 2 * (sum_I partial) / (n_v c); tile rows
// summed in increasing order.  Non-finite results set flag bit 0.
__global__ void __launch_bounds__(64) k_grad_final(int nt, int q,
                                                   const double* partial,
                                                   const double* lam,
                                                   HoldoutNorm hn, double* dlog,
                                                   int* flags) {
  const int64_t m = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= q) return;
  double s = 0.0;
  for (int I = 0; I < nt; ++I) s += partial[(m * nt + I) * q + t];
  const double g = lam[t] * 2.0 * s / hn.count[m];
  dlog[m * q + t] = g;
  if (!isfinite(g)) flags[m * q + t] |= 1;
}

hipError_t launch_trmv_interp(int64_t d, int nmat, int M, int q, int c,
                              int64_t ldz, const double* theta_t,
                              const double* w_dev, const double* X, double* Out,
                              hipStream_t s) {
  const int nt = (int)ntiles_of(d);
  const int64_t dp = (int64_t)nt * NB;
  const int ncb = (int)(ldz / NB);
  PICHOL_LAUNCH(k_trmv_interp, dim3((unsigned)(ncb * nt * nmat)), dim3(256), 0,
                s, dp, nt, theta_t, packed_elems_of(d), M, q, c, ldz, ncb,
                w_dev, X, Out);
  return hipGetLastError();
}

hipError_t launch_grad_dot(int64_t d, int nmat, int q, int c, int64_t ldz,
                           const double* x1, const double* y1,
                           const double* x2, const double* y2,
                           const double* lam_dev, const HoldoutNorm& hn,
                           double* partial, double* dlog, int* flags,
                           hipStream_t s) {
  const int nt = (int)ntiles_of(d);
  PICHOL_LAUNCH(k_grad_partial, dim3((unsigned)nt, (unsigned)nmat), dim3(256), 0,
                s, nt, q, c, ldz, x1, y1, x2, y2, partial);
  PICHOL_LAUNCH(k_grad_final, dim3((unsigned)((q + 63) / 64), (unsigned)nmat),
                dim3(64), 0, s, nt, q, partial, lam_dev, hn, dlog, flags);
  return hipGetLastError();
}

}  // namespace pichol
