// Accuracy diagnostics of the interpolation (the paper's NRMSE section):
// the normalised root-mean-squared error of fitted factors against exact
// ones, and the hold-out NRMSE of the cross-validation errors.  Neither is
// on the timed path; both are reductions in a fixed order (reproducible).
#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

// Pairwise combination of (count, mean, sum of squared deviations) of two
// sets (Chan, Golub and LeVeque's update).
__device__ inline void merge_stats(double& n, double& mean, double& m2,
                                   double nb, double meanb, double m2b) {
  if (nb == 0.0) return;
  if (n == 0.0) {
    n = nb;
    mean = meanb;
    m2 = m2b;
    return;
  }
  const double nn = n + nb, delta = meanb - mean;
  mean += delta * (nb / nn);
  m2 += m2b + delta * delta * (n * nb / nn);
  n = nn;
}

// Tile (I,J) of matrix m: over its entries (i, j) with j <= i < d, the
// count, mean and squared deviations of L (each thread walks its strided
// entries in order, then a fixed tree over the 256 threads) and the sum of
// (Lhat - L)^2.  part[(m * ntile + tile) * 4 + 0..3].
__global__ void __launch_bounds__(256) k_nrmse_partial(int64_t d, int64_t S,
                                                       const double* Lhat,
                                                       const double* L,
                                                       double* part) {
  __shared__ double sn[256], smean[256], sm2[256], ssd[256];
  const int tile = blockIdx.x;
  const int64_t m = blockIdx.y;
  const int ntile = gridDim.x;
  const int I = tri_row(tile), J = tile - (int)tri(I);
  const double* a = L + m * S + tile_off(I, J);
  const double* ah = Lhat + m * S + tile_off(I, J);
  const int tid = threadIdx.x;
  double n = 0.0, mean = 0.0, m2 = 0.0, sd = 0.0;
  for (int e = tid; e < NB2; e += 256) {
    const int64_t i = (int64_t)I * NB + (e & (NB - 1));
    const int64_t j = (int64_t)J * NB + (e >> 7);
    if (i >= d || j > i) continue;
    const double v = a[e], dv = ah[e] - v;
    sd += dv * dv;
    n += 1.0;
    const double delta = v - mean;
    mean += delta / n;
    m2 += delta * (v - mean);
  }
  sn[tid] = n;
  smean[tid] = mean;
  sm2[tid] = m2;
  ssd[tid] = sd;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      double n0 = sn[tid], mu0 = smean[tid], q0 = sm2[tid];
      merge_stats(n0, mu0, q0, sn[tid + w], smean[tid + w], sm2[tid + w]);
      sn[tid] = n0;
      smean[tid] = mu0;
      sm2[tid] = q0;
      ssd[tid] += ssd[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* o = part + (m * ntile + tile) * 4;
    o[0] = sn[0];
    o[1] = smean[0];
    o[2] = sm2[0];
    o[3] = ssd[0];
  }
}

// out[m] = sqrt(sum (Lhat - L)^2) / sqrt(sum (L - mean L)^2), the tiles'
// statistics merged in tile order.
__global__ void __launch_bounds__(64) k_nrmse_final(int ntile, int nmat,
                                                    const double* part,
                                                    double* out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nmat) return;
  double n = 0.0, mean = 0.0, m2 = 0.0, sd = 0.0;
  for (int t = 0; t < ntile; ++t) {
    const double* p = part + ((int64_t)m * ntile + t) * 4;
    merge_stats(n, mean, m2, p[0], p[1], p[2]);
    sd += p[3];
  }
  out[m] = sqrt(sd) / sqrt(m2);
}

hipError_t launch_factor_nrmse(int64_t d, int nmat, const double* Lhat,
                               const double* L, double* part, double* out,
                               hipStream_t s) {
  const int nt = (int)ntiles_of(d);
  const int ntile = (int)tri(nt);
  PICHOL_LAUNCH(k_nrmse_partial, dim3((unsigned)ntile, (unsigned)nmat),
                dim3(256), 0, s, d, packed_elems_of(d), Lhat, L, part);
  PICHOL_LAUNCH(k_nrmse_final, dim3((unsigned)((nmat + 63) / 64)), dim3(64), 0,
                s, ntile, nmat, part, out);
  return hipGetLastError();
}

// Sum over the 256 threads of v, in a fixed tree; every thread gets the
// total.  Uses red[256]; ends with a barrier.
__device__ inline double block_sum(double v, double* red, int tid) {
  red[tid] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

// Fold f = blockIdx.x: SST_f = sum over its validation rows and the c
// columns of (Y - column mean)^2 (two passes per column, columns in
// order); then nrmse[f*q + t] = sqrt(err[f*q + t] * n_v * c / SST_f).
__global__ void __launch_bounds__(256) k_holdout_nrmse(FoldSplit fs, int c,
                                                       int q, const double* Y,
                                                       int64_t ldy,
                                                       const double* err,
                                                       double* nrmse) {
  __shared__ double red[256];
  const int f = blockIdx.x, tid = threadIdx.x;
  const int64_t r0 = fs.start[f], r1 = fs.start[f + 1], nv = r1 - r0;
  double sst = 0.0;
  for (int cc = 0; cc < c; ++cc) {
    double s = 0.0;
    for (int64_t r = r0 + tid; r < r1; r += 256) s += Y[r * ldy + cc];
    const double mean = block_sum(s, red, tid) / (double)nv;
    double ss = 0.0;
    for (int64_t r = r0 + tid; r < r1; r += 256) {
      const double dv = Y[r * ldy + cc] - mean;
      ss += dv * dv;
    }
    sst += block_sum(ss, red, tid);
  }
  const double scale = (double)nv * (double)c / sst;
  for (int t = tid; t < q; t += 256)
    nrmse[(int64_t)f * q + t] = sqrt(err[(int64_t)f * q + t] * scale);
}

hipError_t launch_holdout_nrmse(const FoldSplit& fs, int c, int q,
                                const double* Y, int64_t ldy,
                                const double* err, double* nrmse,
                                hipStream_t s) {
  PICHOL_LAUNCH(k_holdout_nrmse, dim3((unsigned)fs.k), dim3(256), 0, s, fs, c,
                q, Y, ldy, err, nrmse);
  return hipGetLastError();
}

}  // namespace pichol
