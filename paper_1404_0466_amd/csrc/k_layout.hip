// Conversions between dense row-major matrices, the tile-packed triangle
// and the right-hand-side slab.  These are data-movement kernels for the
// library's users and tests, not part of the timed path.
#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

// One block per (matrix, tile); thread e walks the tile in storage order
// (column-major), so packed writes are coalesced.
__global__ void __launch_bounds__(256) k_pack(int64_t d, const double* A,
                                              int64_t lda, double* P,
                                              int64_t S) {
  const int64_t mat = blockIdx.y;
  const int tile = blockIdx.x;
  const int I = tri_row(tile), J = tile - (int)tri(I);
  const double* a = A + mat * lda * d;
  double* p = P + mat * S + tile_off(I, J);
  for (int e = threadIdx.x; e < NB2; e += blockDim.x) {
    const int64_t i = (int64_t)I * NB + (e & (NB - 1));
    const int64_t j = (int64_t)J * NB + (e >> 7);
    double v;
    if (i >= d || j >= d)
      v = (i == j) ? 1.0 : 0.0;
    else
      v = (i >= j) ? a[i * lda + j] : 0.0;
    p[e] = v;
  }
}

__global__ void __launch_bounds__(256) k_unpack(int64_t d, const double* P,
                                                int64_t S, double* A,
                                                int64_t lda) {
  const int64_t mat = blockIdx.y;
  const int64_t i = blockIdx.x;
  const double* p = P + mat * S;
  double* a = A + mat * lda * d + i * lda;
  const int I = (int)(i / NB), ii = (int)(i % NB);
  for (int64_t j = threadIdx.x; j < d; j += blockDim.x) {
    double v = 0.0;
    if (j <= i) {
      const int J = (int)(j / NB), jj = (int)(j % NB);
      v = p[tile_off(I, J) + (int64_t)jj * NB + ii];
    }
    a[j] = v;
  }
}

// W[m][t][i][j] = Z[m][i][t*c + j]
__global__ void __launch_bounds__(256) k_slab_to_weights(int64_t d, int q,
                                                         int c, int64_t ldz,
                                                         int64_t dp,
                                                         const double* Z,
                                                         double* W) {
  const int64_t mat = blockIdx.z;
  const int t = blockIdx.y;
  const int64_t n = d * c;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / c, j = e % c;
    W[((mat * q + t) * d) * c + e] = Z[(mat * dp + i) * ldz + (int64_t)t * c + j];
  }
}

// Small host arrays (lambda values) reach the device as kernel arguments,
// which are captured at launch: the host buffer may be released as soon as
// the launch call returns, and the copy is stream-ordered.
struct DoubleChunk {
  int n;
  double v[256];
};

__global__ void k_store_doubles(DoubleChunk ch, double* dst) {
  const int i = threadIdx.x;
  if (i < ch.n) dst[i] = ch.v[i];
}

hipError_t launch_store_doubles(const double* host, int n, double* dev,
                                hipStream_t s) {
  for (int o = 0; o < n; o += 256) {
    DoubleChunk ch;
    ch.n = (n - o) < 256 ? (n - o) : 256;
    for (int i = 0; i < ch.n; ++i) ch.v[i] = host[o + i];
    PICHOL_LAUNCH(k_store_doubles, dim3(1), dim3(256), 0, s, ch, dev + o);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pack(int64_t d, int nmat, const double* A, int64_t lda,
                       double* P, hipStream_t s) {
  const int64_t nt = ntiles_of(d);
  dim3 grid((unsigned)tri(nt), (unsigned)nmat);
  PICHOL_LAUNCH(k_pack, grid, dim3(256), 0, s, d, A, lda, P,
                     packed_elems_of(d));
  return hipGetLastError();
}

hipError_t launch_unpack(int64_t d, int nmat, const double* P, double* A,
                         int64_t lda, hipStream_t s) {
  dim3 grid((unsigned)d, (unsigned)nmat);
  PICHOL_LAUNCH(k_unpack, grid, dim3(256), 0, s, d, P,
                     packed_elems_of(d), A, lda);
  return hipGetLastError();
}

hipError_t launch_slab_to_weights(int64_t d, int nmat, int q, int c,
                                  int64_t ldz, const double* Z, double* W,
                                  hipStream_t s) {
  const int64_t n = d * c;
  unsigned bx = (unsigned)((n + 255) / 256);
  if (bx > 4096) bx = 4096;
  dim3 grid(bx, (unsigned)q, (unsigned)nmat);
  PICHOL_LAUNCH(k_slab_to_weights, grid, dim3(256), 0, s, d, q, c, ldz,
                     ntiles_of(d) * NB, Z, W);
  return hipGetLastError();
}

// dst[i] = src[i] (int32), through vector stores: gathers per-problem
// status words out of a batch's stacked arrays.
__global__ void __launch_bounds__(256) k_copy_i32(int64_t n, const int* src,
                                                  int* dst) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

hipError_t launch_copy_i32(int64_t n, const int* src, int* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t bx = (n + 255) / 256;
  if (bx > 1024) bx = 1024;
  PICHOL_LAUNCH(k_copy_i32, dim3((unsigned)bx), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

// ---- vectorisations of a factor (Sec. 5), for the layout comparison.
// Position of lower entry (i, j) of an order-h triangle in the recursive
// vectorisation of Sec. 5 (eq. recursive): the triangle is split at
// half = h/2 into the square block L12 (rows half.., columns ..half),
// stored first in row-major order, then the triangle L11, then the triangle
// L22, each vectorised the same way until the order is at most h0, where
// rows are concatenated.  (h need not be a power of two: L12 is then
// (h - half) x half.)
__device__ inline int64_t recursive_pos(int64_t i, int64_t j, int64_t h,
                                        int64_t h0) {
  int64_t base = 0;
  while (h > h0) {
    const int64_t half = h / 2, rest = h - half;
    if (i >= half && j < half) return base + (i - half) * half + j;
    if (i < half) {
      base += rest * half;
      h = half;
    } else {
      base += rest * half + half * (half + 1) / 2;
      i -= half;
      j -= half;
      h = rest;
    }
  }
  return base + i * (i + 1) / 2 + j;
}

// One 128 x 128 tile (I,J) of a tile-packed factor into a vectorised
// layout: the tile is read column-major (coalesced) into LDS and written
// row by row, so the writes of a row segment are contiguous in the
// row-wise, full-matrix and (within its blocks) recursive orders.  For the
// full-matrix layout the tiles above the diagonal are written as zeros.
__global__ void __launch_bounds__(256) k_vectorize(int64_t d, int64_t S,
                                                   const double* P, int layout,
                                                   int64_t h0, int64_t N,
                                                   double* T) {
  __shared__ double lds[NB * LDS_LD];
  const int64_t nt = ntiles_of(d);
  const int64_t mat = blockIdx.y;
  const int I = (int)(blockIdx.x / nt), J = (int)(blockIdx.x % nt);
  const int tid = threadIdx.x;
  double* out = T + mat * N;
  if (J > I) {
    if (layout != 2) return;
    for (int e = tid; e < NB2; e += blockDim.x) {
      const int64_t i = (int64_t)I * NB + (e >> 7), j = (int64_t)J * NB + (e & (NB - 1));
      if (i < d && j < d) out[i * d + j] = 0.0;
    }
    return;
  }
  const double* tile = P + mat * S + tile_off(I, J);
  for (int e = tid; e < NB2; e += blockDim.x)
    lds[(e >> 7) * LDS_LD + (e & (NB - 1))] = tile[e];  // lds[col][row]
  __syncthreads();
  for (int e = tid; e < NB2; e += blockDim.x) {
    const int r = e >> 7, cc = e & (NB - 1);
    const int64_t i = (int64_t)I * NB + r, j = (int64_t)J * NB + cc;
    if (i >= d || j >= d) continue;
    const double v = lds[cc * LDS_LD + r];
    if (layout == 2) {
      out[i * d + j] = j <= i ? v : 0.0;
    } else if (j <= i) {
      out[layout == 1 ? i * (i + 1) / 2 + j : recursive_pos(i, j, d, h0)] = v;
    }
  }
}

hipError_t launch_vectorize(int64_t d, int nmat, const double* P, int layout,
                            int64_t h0, int64_t N, double* T, hipStream_t s) {
  const int64_t nt = ntiles_of(d);
  PICHOL_LAUNCH(k_vectorize, dim3((unsigned)(nt * nt), (unsigned)nmat),
                dim3(256), 0, s, d, packed_elems_of(d), P, layout, h0, N, T);
  return hipGetLastError();
}

}  // namespace pichol
