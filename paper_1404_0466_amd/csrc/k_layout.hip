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

}  // namespace pichol
