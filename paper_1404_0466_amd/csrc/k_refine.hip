// Iterative refinement of the solves (residual correction).
//
// With Z holding the solutions W_t of every (fold, lambda) in the slab
// layout, one refinement step is
//     R_t = B_f - (H_f + lambda_t I) W_t        (FP64)
//     solve Lhat_t Lhat_t^T D_t = R_t            (the same factors, in place)
//     W_t += D_t
// The residual of all q values of a fold is one product of the symmetric
// H_f (full 128 x 128 tiles, both triangles) with the slab, on FP64 MFMA;
// the shift and B enter as the accumulators' starting values.
#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

// Full-tile H_f = scale_f * sum_{b != f} G_b for every tile (I,J) of the
// nt x nt grid (fold-block sums in increasing block order, as for the packed
// lower triangle, so the lower tiles agree with it bit for bit); entries
// outside the first d rows/columns are 0.  Output tile (I,J) of fold f at
// ((f*nt + I)*nt + J) * 16384, column-major.
__global__ void __launch_bounds__(256) k_full_h(int64_t d, int nt, FoldSplit fs,
                                                const double* G, double* Hf) {
  const int f = blockIdx.y;
  const int I = blockIdx.x / nt, J = blockIdx.x - (blockIdx.x / nt) * nt;
  const double sc = fs.scale[f];
  const int64_t gstride = (int64_t)nt * nt * NB2;
  const double* g0 = G + ((int64_t)I * nt + J) * NB2;
  double* h = Hf + (((int64_t)f * nt + I) * nt + J) * NB2;
  for (int e = threadIdx.x; e < NB2; e += blockDim.x) {
    const int64_t i = (int64_t)I * NB + (e & (NB - 1));
    const int64_t j = (int64_t)J * NB + (e >> 7);
    double v = 0.0;
    if (i < d && j < d) {
      double acc = 0.0;
      for (int b = 0; b < fs.k; ++b)
        if (b != f) acc += g0[b * gstride + e];
      v = acc * sc;
    }
    h[e] = v;
  }
}

// R[m] rows of tile I, slab columns of block cb:
//   R = B_rep - lambda_col * Z_I - sum_J H_f(I,J) Z_J,
// where B_rep holds column col % c of B_m for col < q*c (0 beyond) and
// lambda_col = lam[col / c].  The four waves of a workgroup own 64 x 64
// quarters of the 128 x 128 output block; products run over the nt
// 128-row blocks of Z.  Logical workgroup ids run over column blocks
// fastest, so the blocks that read the same H tiles meet on one XCD.
__global__ void __launch_bounds__(256) k_residual(int64_t dp, int nt, int q,
                                                  int c, int64_t ldz, int ncb,
                                                  const double* Hf,
                                                  const double* B,
                                                  const double* lam,
                                                  const double* Z, double* R) {
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int cb = id % ncb;
  const int rest = id / ncb;
  const int I = rest % nt;
  const int64_t m = rest / nt;
  const int w = threadIdx.x >> 6, wi = w >> 1, wj = w & 1;
  const LaneXY lx;
  const int64_t col = (int64_t)cb * NB + wj * 64 + lx.col0();
  const int64_t qc = (int64_t)q * c;
  v4d lam4;
  int bc[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const bool ok = (col + e) < qc;
    lam4[e] = ok ? lam[(col + e) / c] : 0.0;
    bc[e] = ok ? (int)((col + e) % c) : -1;
  }
  const int64_t row0 = m * dp + (int64_t)I * NB + wi * 64;
  Acc64 acc;
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const int64_t row = row0 + lx.row(v, bi);
      const v4d z = ld4(Z + row * ldz + col);
      v4d b;
#pragma unroll
      for (int e = 0; e < 4; ++e) b[e] = bc[e] >= 0 ? B[row * c + bc[e]] : 0.0;
      acc.set_row(v, bi, b - lam4 * z);
    }
  const v4d neg = {-1.0, -1.0, -1.0, -1.0};
  const double* hrow = Hf + (m * nt + I) * (int64_t)nt * NB2 + wi * 64;
  const double* zb = Z + m * dp * ldz + (int64_t)cb * NB + wj * 64;
  for (int J = 0; J < nt; ++J)
    mma_panel_scaled(acc, hrow + (int64_t)J * NB2, NB,
                     zb + (int64_t)J * NB * ldz, ldz, NB, neg);
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
      st4(R + (row0 + lx.row(v, bi)) * ldz + col, acc.row(v, bi));
}

// Z += D over n elements (n a multiple of 4).
__global__ void __launch_bounds__(256) k_slab_add(int64_t n4, const double* D,
                                                  double* Z) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n4;
       e += (int64_t)gridDim.x * blockDim.x)
    st4(Z + 4 * e, ld4(Z + 4 * e) + ld4(D + 4 * e));
}

hipError_t launch_full_h(int64_t d, const FoldSplit& fs, const double* G,
                         double* Hf, hipStream_t s) {
  const int nt = (int)ntiles_of(d);
  PICHOL_LAUNCH(k_full_h, dim3((unsigned)(nt * nt), (unsigned)fs.k), dim3(256),
                0, s, d, nt, fs, G, Hf);
  return hipGetLastError();
}

hipError_t launch_residual(int64_t d, int nmat, int q, int c, int64_t ldz,
                           const double* Hf, const double* B,
                           const double* lam_dev, const double* Z, double* R,
                           hipStream_t s) {
  const int nt = (int)ntiles_of(d);
  const int64_t dp = (int64_t)nt * NB;
  const int ncb = (int)(ldz / NB);
  PICHOL_LAUNCH(k_residual, dim3((unsigned)(ncb * nt * nmat)), dim3(256), 0, s,
                dp, nt, q, c, ldz, ncb, Hf, B, lam_dev, Z, R);
  return hipGetLastError();
}

hipError_t launch_slab_add(int64_t d, int nmat, int64_t ldz, const double* D,
                           double* Z, hipStream_t s) {
  const int64_t n4 = (int64_t)nmat * ntiles_of(d) * NB * ldz / 4;
  int64_t bx = (n4 + 255) / 256;
  if (bx > 4096) bx = 4096;
  PICHOL_LAUNCH(k_slab_add, dim3((unsigned)bx), dim3(256), 0, s, n4, D, Z);
  return hipGetLastError();
}

}  // namespace pichol
