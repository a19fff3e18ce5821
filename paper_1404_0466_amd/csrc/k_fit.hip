// Least-squares fit of every factor entry (Algorithm 1 steps 2-6) and
// evaluation of the fitted factor (Sec. 3.3).
//
// Algorithm 1 stacks the g sample factors as the rows of T and solves the
// normal equations for Theta.  Here the packed factors already are the
// rows of T (the tile-packed triangle is the vectorisation), and Theta is
// formed as P T with P = V^+ computed once on the host.  The inner dimension
// is g, so both kernels stream memory: one read of every sample entry, one
// write of every coefficient.
#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

// Theta(m, p) tile (I,J) = sum_s P[p][s] L(m, s) tile (I,J); also written
// with the tile stored row-major into theta_t (when non-null).  The grid
// covers the tiles of columns J0, J0+1, ... column by column (each column J
// holds the tiles I = J .. nt-1).
template <int M>
__global__ void __launch_bounds__(256) k_fit(int64_t S, FitCoef fc,
                                             const double* L, double* theta,
                                             double* theta_t, int nt, int J0) {
  __shared__ double lds[16 * LDS_LD];
  const int64_t m = blockIdx.y;
  int J = J0, I = blockIdx.x;
  while (I >= nt - J) {
    I -= nt - J;
    ++J;
  }
  I += J;
  const int64_t toff = tile_off(I, J);
  const int g = fc.g;
  const int tid = threadIdx.x;
  // the tile in eight chunks of 16 columns; each thread owns two runs of
  // four consecutive entries of a chunk (32-byte loads and stores)
  for (int cb = 0; cb < NB / 16; ++cb) {
    v4d th[2][M];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int p = 0; p < M; ++p) th[h][p] = v4d{0.0, 0.0, 0.0, 0.0};
    const int64_t base = toff + cb * 16 * NB;
    for (int s = 0; s < g; ++s) {
      const double* src = L + (m * g + s) * S + base;
      const v4d x0 = ld4(src + 4 * tid), x1 = ld4(src + 4 * (tid + 256));
#pragma unroll
      for (int p = 0; p < M; ++p) {
        th[0][p] += fc.P[p][s] * x0;
        th[1][p] += fc.P[p][s] * x1;
      }
    }
#pragma unroll
    for (int p = 0; p < M; ++p) {
      double* dst = theta + (m * M + p) * S + base;
      st4(dst + 4 * tid, th[0][p]);
      st4(dst + 4 * (tid + 256), th[1][p]);
    }
    if (theta_t == nullptr) continue;
#pragma unroll
    for (int p = 0; p < M; ++p) {
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = 4 * (tid + 256 * h);  // within the chunk
        const int col = e >> 7, row = e & (NB - 1);
#pragma unroll
        for (int x = 0; x < 4; ++x) lds[col * LDS_LD + row + x] = th[h][p][x];
      }
      __syncthreads();
      double* dst = theta_t + (m * M + p) * S + toff + cb * 16;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = tid + 256 * u;
        const int a = e >> 4, bl = e & 15;
        dst[a * NB + bl] = lds[bl * LDS_LD + a];
      }
    }
  }
}

// Lhat(m, t) = sum_p tau_t^p Theta(m, p), four entries per thread.
__global__ void __launch_bounds__(256) k_eval(int64_t S, int M,
                                              const double* theta,
                                              int nlam, const double* tau,
                                              double* Lhat) {
  const int64_t m = blockIdx.z;
  const int t = blockIdx.y;
  const double tv = tau[t];
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e < S;
       e += (int64_t)gridDim.x * blockDim.x * 4) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    double pw = 1.0;
    for (int p = 0; p < M; ++p) {
      acc += pw * ld4(theta + (m * M + p) * S + e);
      pw *= tv;
    }
    st4(Lhat + (m * nlam + t) * S + e, acc);
  }
}

hipError_t launch_fit_cols(int64_t d, int nmat, const FitCoef& fc,
                           const double* L, double* theta, double* theta_t,
                           int J0, int J1, hipStream_t s) {
  const int nt = (int)ntiles_of(d);
  const int64_t S = packed_elems_of(d);
  if (J0 < 0 || J1 > nt || J0 > J1) return hipErrorInvalidValue;
  // tiles of columns J0 .. J1-1
  const int64_t ntile = tri(nt - J0) - tri(nt - J1);
  if (ntile == 0) return hipSuccess;
  dim3 grid((unsigned)ntile, (unsigned)nmat);
  switch (fc.m) {
#define PICHOL_FIT_CASE(MM)                                                   \
  case MM:                                                                    \
    PICHOL_LAUNCH(k_fit<MM>, grid, dim3(256), 0, s, S, fc, L, theta,          \
                  theta_t, nt, J0);                                           \
    break;
    PICHOL_FIT_CASE(1)
    PICHOL_FIT_CASE(2)
    PICHOL_FIT_CASE(3)
    PICHOL_FIT_CASE(4)
    PICHOL_FIT_CASE(5)
    PICHOL_FIT_CASE(6)
    PICHOL_FIT_CASE(7)
    PICHOL_FIT_CASE(8)
#undef PICHOL_FIT_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fit(int64_t d, int nmat, const FitCoef& fc, const double* L,
                      double* theta, double* theta_t, hipStream_t s) {
  return launch_fit_cols(d, nmat, fc, L, theta, theta_t, 0,
                         (int)ntiles_of(d), s);
}

hipError_t launch_eval(int64_t d, int nmat, int m, const double* theta,
                       int nlam, const double* tau_dev, double* Lhat,
                       hipStream_t s) {
  const int64_t S = packed_elems_of(d);
  unsigned bx = (unsigned)((S / 4 + 255) / 256);
  if (bx > 1024) bx = 1024;
  PICHOL_LAUNCH(k_eval, dim3(bx, (unsigned)nlam, (unsigned)nmat),
                     dim3(256), 0, s, S, m, theta, nlam, tau_dev, Lhat);
  return hipGetLastError();
}

// The hold-out-error variant of Algorithm 1 (PINRMSE): the g-vector of
// exact hold-out errors of fold m at the samples takes the place of T, so
// the fitted coefficients are theta_j = sum_s P[j][s] e[m][s] and the curve
// at grid value t is sum_j tau_t^j theta_j.
__global__ void __launch_bounds__(64) k_pinrmse(FitCoef fc, int q,
                                                const double* tau,
                                                const double* es,
                                                double* err) {
  const int64_t m = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= q) return;
  double th[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double acc = 0.0;
    if (j < fc.m)
      for (int s = 0; s < fc.g; ++s) acc += fc.P[j][s] * es[m * fc.g + s];
    th[j] = acc;
  }
  double out = 0.0, pw = 1.0;
  const double tv = tau[t];
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < fc.m) {
      out += pw * th[j];
      pw *= tv;
    }
  err[m * q + t] = out;
}

hipError_t launch_pinrmse(int nmat, const FitCoef& fc, int q,
                          const double* tau_dev, const double* es, double* err,
                          hipStream_t s) {
  PICHOL_LAUNCH(k_pinrmse, dim3((unsigned)((q + 63) / 64), (unsigned)nmat),
                dim3(64), 0, s, fc, q, tau_dev, es, err);
  return hipGetLastError();
}

// Theta(m, p) = sum_s P[p][s] T(m, s) over flat vectors of length N
// (N a multiple of 4), four entries per thread: the fit on any
// vectorisation of the factors (the layout comparison).
template <int M>
__global__ void __launch_bounds__(256) k_fit_flat(int64_t N, FitCoef fc,
                                                  const double* T,
                                                  double* theta) {
  const int64_t m = blockIdx.y;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; e < N;
       e += (int64_t)gridDim.x * blockDim.x * 4) {
    v4d th[M];
#pragma unroll
    for (int p = 0; p < M; ++p) th[p] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < fc.g; ++s) {
      const v4d t = ld4(T + (m * fc.g + s) * N + e);
#pragma unroll
      for (int p = 0; p < M; ++p) th[p] += fc.P[p][s] * t;
    }
#pragma unroll
    for (int p = 0; p < M; ++p) st4(theta + (m * M + p) * N + e, th[p]);
  }
}

hipError_t launch_fit_flat(int64_t N, int nmat, const FitCoef& fc,
                           const double* T, double* theta, hipStream_t s) {
  int64_t bx = (N / 4 + 255) / 256;
  if (bx > 2048) bx = 2048;
  dim3 grid((unsigned)bx, (unsigned)nmat);
  switch (fc.m) {
#define PICHOL_FITF_CASE(MM)                                                  \
  case MM:                                                                    \
    PICHOL_LAUNCH(k_fit_flat<MM>, grid, dim3(256), 0, s, N, fc, T, theta);    \
    break;
    PICHOL_FITF_CASE(1)
    PICHOL_FITF_CASE(2)
    PICHOL_FITF_CASE(3)
    PICHOL_FITF_CASE(4)
    PICHOL_FITF_CASE(5)
    PICHOL_FITF_CASE(6)
    PICHOL_FITF_CASE(7)
    PICHOL_FITF_CASE(8)
#undef PICHOL_FITF_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_eval_flat(int64_t N, int nmat, int m, const double* theta,
                            int nlam, const double* tau_dev, double* out,
                            hipStream_t s) {
  unsigned bx = (unsigned)((N / 4 + 255) / 256);
  if (bx > 1024) bx = 1024;
  PICHOL_LAUNCH(k_eval, dim3(bx, (unsigned)nlam, (unsigned)nmat), dim3(256), 0,
                s, N, m, theta, nlam, tau_dev, out);
  return hipGetLastError();
}

}  // namespace pichol
