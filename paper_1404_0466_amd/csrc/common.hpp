// Internal definitions shared by the gfx950 kernels of the piCholesky
// library: tile geometry of the packed layout, the FP64 MFMA micro-kernel,
// and launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace pichol {

constexpr int NB = 128;          // tile edge
constexpr int NB2 = NB * NB;     // elements per tile
constexpr int LDS_LD = NB + 1;   // padded leading dimension of LDS tiles

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

__host__ __device__ inline int64_t tri(int64_t I) { return I * (I + 1) / 2; }

// Element offset of tile (I,J), J <= I, inside one packed triangle.
__host__ __device__ inline int64_t tile_off(int64_t I, int64_t J) {
  return (tri(I) + J) * (int64_t)NB2;
}

__host__ __device__ inline int64_t ntiles_of(int64_t d) {
  return (d + NB - 1) / NB;
}

__host__ __device__ inline int64_t packed_elems_of(int64_t d) {
  return d < 1 ? 0 : tri(ntiles_of(d)) * (int64_t)NB2;
}

// Row index r of linear index t in a triangle enumerated row by row
// (t = r(r+1)/2 + col, 0 <= col <= r).
__device__ inline int tri_row(int t) {
  int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (tri(r + 1) <= t) ++r;
  while (tri(r) > t) --r;
  return r;
}

__device__ inline v4d ld4(const double* p) { return *(const v4d*)p; }

// base + e elements, with the offset formed as a 32-bit byte count: a
// wave-uniform base plus a per-lane offset below 4 GiB, the form of the
// scalar-base, 32-bit-offset global addressing mode.
template <typename T>
__device__ inline T* at_elem(T* base, unsigned e) {
  typedef typename std::conditional<std::is_const<T>::value, const char, char>::type B;
  return reinterpret_cast<T*>(reinterpret_cast<B*>(base) + e * (unsigned)sizeof(T));
}
__device__ inline void st4(double* p, v4d v) { *(v4d*)p = v; }

// ---------------------------------------------------------------------------
// FP64 MFMA micro-kernel for one 64 x 64 block per wavefront.
//
// v_mfma_f64_16x16x4f64 computes D(16x16) += A(16x4) B(4x16); lane l
// supplies A[l%16][l/16] and B[l/16][l%16] and holds D[4v + l/16][l%16] in
// element v of its accumulator (checked on gfx950).
//
// The wave's block is the product D'(i,j) = sum_k A'(i,k) B'(k,j) for
// i, j in [0,64).  Operands are read from memory where the non-k index is
// contiguous: A'(i,k) at a[k*lda + i], B'(k,j) at b[k*ldb + j].  To read each
// operand with one 32-byte load per lane and k-step, MFMA block bi takes the
// rows i = 4*(l%16) + bi, and block bj the columns j = 4*(l%16) + bj: lane l
// loads the four consecutive values a[k*lda + 4*(l%16) .. +3] and uses one
// in each block.  Accumulator acc[bi][bj] element v of lane l then holds
//     D'(i = 16*v + 4*(l/16) + bi,  j = 4*(l%16) + bj)
// so the four bj accumulators of a lane are four consecutive j: the
// epilogue writes them with one 32-byte store.
// ---------------------------------------------------------------------------
struct Acc64 {
  // Global row (within the 64-row block) of accumulator element v of block
  // bi for a lane with l/16 = lq: element v holds D[4v + l/16][l%16].
  __device__ static inline int row_of(int lq, int v, int bi) {
    return 16 * v + 4 * lq + bi;
  }
  v4d c[4][4];
  __device__ inline void zero() {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) c[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  __device__ inline void mma(const v4d& a, const v4d& b) {
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        c[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj],
                                                          c[bi][bj], 0, 0, 0);
  }
  // Set row i = 16*v + 4*(l/16) + bi at columns 4*(l%16) .. +3.
  __device__ inline void set_row(int v, int bi, const v4d& x) {
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) c[bi][bj][v] = x[bj];
  }
  // Values of row i = 16*v + 4*(l/16) + bi at columns 4*(l%16) .. +3.
  __device__ inline v4d row(int v, int bi) const {
    return v4d{c[bi][0][v], c[bi][1][v], c[bi][2][v], c[bi][3][v]};
  }
};

// acc += sum over k in [0,K) of A'(i,k) B'(k,j); K a multiple of 4.
// a, b point at A'(0,0) and B'(0,0) of the wave's block.
__device__ inline void mma_panel(Acc64& acc, const double* a, int64_t lda,
                                 const double* b, int64_t ldb, int K) {
  const int l = threadIdx.x & 63;
  const double* pa = a + (int64_t)(l >> 4) * lda + 4 * (l & 15);
  const double* pb = b + (int64_t)(l >> 4) * ldb + 4 * (l & 15);
  const int64_t sa = 4 * lda, sb = 4 * ldb;
  v4d av = ld4(pa), bv = ld4(pb);
  for (int k0 = 4; k0 < K; k0 += 4) {
    pa += sa;
    pb += sb;
    v4d an = ld4(pa), bn = ld4(pb);
    acc.mma(av, bv);
    av = an;
    bv = bn;
  }
  acc.mma(av, bv);
}

// The same 64 x 64 wave block on FP32 MFMA.  v_mfma_f32_16x16x4f32 takes
// its operands in the lane layout of the FP64 instruction, but element v of
// lane l holds D[4(l/16) + v][l%16] (four consecutive rows per lane), so
// the global row of (v, bi) is 16(l/16) + 4v + bi.  FP64 operands are
// rounded to FP32 as they are loaded, products accumulate in FP32, and rows
// are handed back in FP64.
struct Acc64F {
  __device__ static inline int row_of(int lq, int v, int bi) {
    return 16 * lq + 4 * v + bi;
  }
  v4f c[4][4];
  __device__ inline void zero() {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) c[i][j] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  }
  __device__ inline void mma(const v4f& a, const v4f& b) {
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        c[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bi], b[bj],
                                                          c[bi][bj], 0, 0, 0);
  }
  __device__ inline v4d row(int v, int bi) const {
    return v4d{(double)c[bi][0][v], (double)c[bi][1][v], (double)c[bi][2][v],
               (double)c[bi][3][v]};
  }
};

__device__ inline v4f to_f32(const v4d& x) {
  return v4f{(float)x[0], (float)x[1], (float)x[2], (float)x[3]};
}

__device__ inline void mma_panel_f32(Acc64F& acc, const double* a, int64_t lda,
                                     const double* b, int64_t ldb, int K) {
  const int l = threadIdx.x & 63;
  const double* pa = a + (int64_t)(l >> 4) * lda + 4 * (l & 15);
  const double* pb = b + (int64_t)(l >> 4) * ldb + 4 * (l & 15);
  const int64_t sa = 4 * lda, sb = 4 * ldb;
  v4d av = ld4(pa), bv = ld4(pb);
  for (int k0 = 4; k0 < K; k0 += 4) {
    pa += sa;
    pb += sb;
    v4d an = ld4(pa), bn = ld4(pb);
    acc.mma(to_f32(av), to_f32(bv));
    av = an;
    bv = bn;
  }
  acc.mma(to_f32(av), to_f32(bv));
}

// acc += sum_k A'(i,k) (scale .* B'(k,j)); scale holds the factor of the
// lane's four columns.
__device__ inline void mma_panel_scaled(Acc64& acc, const double* a,
                                        int64_t lda, const double* b,
                                        int64_t ldb, int K, v4d scale) {
  const int l = threadIdx.x & 63;
  const double* pa = a + (int64_t)(l >> 4) * lda + 4 * (l & 15);
  const double* pb = b + (int64_t)(l >> 4) * ldb + 4 * (l & 15);
  const int64_t sa = 4 * lda, sb = 4 * ldb;
  v4d av = ld4(pa), bv = ld4(pb);
  for (int k0 = 4; k0 < K; k0 += 4) {
    pa += sa;
    pb += sb;
    v4d an = ld4(pa), bn = ld4(pb);
    acc.mma(av, bv * scale);
    av = an;
    bv = bn;
  }
  acc.mma(av, bv * scale);
}

// acc -= sum over k in [0,K) of A'(i,k) B'(k,j) (the A operand negated).
__device__ inline void mma_panel_sub(Acc64& acc, const double* a, int64_t lda,
                                     const double* b, int64_t ldb, int K) {
  const int l = threadIdx.x & 63;
  const double* pa = a + (int64_t)(l >> 4) * lda + 4 * (l & 15);
  const double* pb = b + (int64_t)(l >> 4) * ldb + 4 * (l & 15);
  const int64_t sa = 4 * lda, sb = 4 * ldb;
  v4d av = ld4(pa), bv = ld4(pb);
  for (int k0 = 4; k0 < K; k0 += 4) {
    pa += sa;
    pb += sb;
    v4d an = ld4(pa), bn = ld4(pb);
    acc.mma(-av, bv);
    av = an;
    bv = bn;
  }
  acc.mma(-av, bv);
}

// Workgroups are dispatched to the eight XCDs round-robin by linear id, and
// each XCD has its own L2.  This maps the hardware id to a logical id such
// that every XCD receives one contiguous range of logical ids, so work items
// that share operands (tiles of one matrix) meet in the same L2.
__device__ inline int xcd_remap(int id, int n) {
  const int q = n >> 3, rem = n & 7;
  const int xcd = id & 7, slot = id >> 3;
  return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

// s ~ sqrt(x) and y ~ 1/sqrt(x) for a positive x: the hardware
// reciprocal-square-root estimate refined by two Newton steps
// y <- y + y (1 - x y^2) / 2, then s = x y corrected once by
// s <- s + y (x - s^2) / 2.  A few-ulp replacement for a correctly rounded
// square root followed by divisions, with a much shorter dependency chain;
// a non-positive or NaN x gives non-finite results.
__device__ inline void sqrt_rsqrt(double x, double& s, double& y) {
  double r = __builtin_amdgcn_rsq(x);
  double e = fma(-x * r, r, 1.0);
  r = fma(0.5 * r, e, r);
  e = fma(-x * r, r, 1.0);
  r = fma(0.5 * r, e, r);
  double t = x * r;
  t = fma(0.5 * r, fma(-t, t, x), t);
  s = t;
  y = r;
}

__device__ inline double bcast_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// A 128 x 128 lower-triangular matrix in LDS as its 36 blocks of 16 x 16:
// block (I, J), I >= J, at blk_off(I, J), column-major with a column stride
// of 17 doubles, so a wave reading a block along its columns (MFMA A
// operands) or along its rows (B operands) meets no bank conflicts.  The
// diagonal blocks hold zeros above their diagonal.
constexpr int TLD = 17;
constexpr int TBLK = 16 * TLD;
constexpr int TRI_LDS = 36 * TBLK;  // doubles: 78,336 bytes
__device__ inline int blk_off(int I, int J) { return (I * (I + 1) / 2 + J) * TBLK; }

// acc (a 16 x 16 block in the accumulator layout: element v of lane l is
// D(4v + l/16, l%16)) += A B for two LDS blocks; lane l supplies
// A(l%16, 4s + l/16) and B(4s + l/16, l%16) in step s.
__device__ inline void mfma_blk(v4d& acc, const double* A, const double* B,
                                int lq, int lr) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * s + lq;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[k * TLD + lr], B[lr * TLD + k],
                                               acc, 0, 0, 0);
  }
}

// One level of the blocked inverse: the matrix is split into diagonal
// regions of 2n blocks, each [T11 0; T21 T22] with n x n blocks per part,
// whose parts T11 and T22 already hold their inverses X11, X22.  Then
// T^{-1} = [X11 0; X21 X22] with X21 = -X22 T21 X11, formed in two MFMA
// products: P = T21 X11 overwrites T21, then X21 = -X22 P overwrites P.
// Each output block of each region is one work unit, dealt to the four
// waves in turn; a barrier separates every read of a part from its
// overwrite.
template <int N>
__device__ __forceinline__ void inv_level(double* S, int w, int lq, int lr) {
  constexpr int REG = 8 / (2 * N);         // regions
  constexpr int UNITS = REG * N * N;       // output blocks per product
  constexpr int PER = (UNITS + 3) / 4;     // units per wave
  v4d acc[PER];
  // P(r, c) = sum_{k >= c} T21(r, k) X11(k, c)   (X11 lower triangular)
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int u = w + 4 * j;
    if (u < UNITS) {
      const int g = u / (N * N), r = (u / N) % N, c = u % N;
      const int a0 = 2 * N * g, c0 = a0 + N;
      for (int k = c; k < N; ++k)
        mfma_blk(acc[j], S + blk_off(c0 + r, a0 + k), S + blk_off(a0 + k, a0 + c),
                 lq, lr);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int u = w + 4 * j;
    if (u < UNITS) {
      const int g = u / (N * N), r = (u / N) % N, c = u % N;
      const int a0 = 2 * N * g, c0 = a0 + N;
      double* o = S + blk_off(c0 + r, a0 + c);
#pragma unroll
      for (int v = 0; v < 4; ++v) o[lr * TLD + 4 * v + lq] = acc[j][v];
    }
  }
  __syncthreads();
  // X21(r, c) = -sum_{k <= r} X22(r, k) P(k, c)   (X22 lower triangular)
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int u = w + 4 * j;
    if (u < UNITS) {
      const int g = u / (N * N), r = (u / N) % N, c = u % N;
      const int a0 = 2 * N * g, c0 = a0 + N;
      for (int k = 0; k <= r; ++k)
        mfma_blk(acc[j], S + blk_off(c0 + r, c0 + k), S + blk_off(c0 + k, a0 + c),
                 lq, lr);
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int u = w + 4 * j;
    if (u < UNITS) {
      const int g = u / (N * N), r = (u / N) % N, c = u % N;
      const int a0 = 2 * N * g, c0 = a0 + N;
      double* o = S + blk_off(c0 + r, a0 + c);
#pragma unroll
      for (int v = 0; v < 4; ++v) o[lr * TLD + 4 * v + lq] = -acc[j][v];
    }
  }
  __syncthreads();
}

// Inverts, in place, the lower-triangular matrix held in S (the layout
// above) with the whole 256-thread workgroup; every thread must have
// finished writing S (a barrier) before the call, and S is complete on
// return.
//   1. the eight 16 x 16 diagonal blocks by forward substitution, one
//      column per lane (lanes 0-31 of each wave take two blocks);
//   2. three levels that join inverses of 16, 32 and 64 rows into inverses
//      of 32, 64 and 128 rows on FP64 MFMA (inv_level).
__device__ __forceinline__ void tri_inv_lds(double* S) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int lq = l >> 4, lr = l & 15;
  // 1. diagonal blocks: lane j of the lower or upper 16 lanes of the first
  // half of wave w solves column j of the inverse of block 2w or 2w + 1
  // (entries above the diagonal come out zero; the second half repeats the
  // work and does not store it)
  double xc[16];
  const int hb = 2 * w + ((l >> 4) & 1);
  {
    const double* T = S + blk_off(hb, hb);
    const int j = lr;
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      double s = a == j ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < a; ++k) s -= T[k * TLD + a] * xc[k];
      xc[a] = s / T[a * TLD + a];
      // keep the compiler from hoisting every row's loads at once: row a
      // is complete before the next row's loads (an empty statement that
      // emits no instruction)
      asm volatile("" : "+v"(xc[a]) : : "memory");
    }
  }
  __syncthreads();
  if (l < 32) {
    double* X = S + blk_off(hb, hb) + lr * TLD;
#pragma unroll
    for (int a = 0; a < 16; ++a) X[a] = xc[a];
  }
  __syncthreads();
  // 2. join: 16 -> 32 -> 64 -> 128 rows
  inv_level<1>(S, w, lq, lr);
  inv_level<2>(S, w, lq, lr);
  inv_level<4>(S, w, lq, lr);
}

// Lane coordinates inside a 64 x 64 wave block.
struct LaneXY {
  int lq;  // l / 16
  int lr;  // l % 16
  __device__ inline LaneXY() {
    int l = threadIdx.x & 63;
    lq = l >> 4;
    lr = l & 15;
  }
  __device__ inline int row(int v, int bi) const { return 16 * v + 4 * lq + bi; }
  __device__ inline int col0() const { return 4 * lr; }
};

}  // namespace pichol
