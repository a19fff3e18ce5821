// Batched Cholesky factorization of shifted matrices H + lambda I
// (Sec. 3.2; Algorithm 1 step 1 and the exact per-lambda baseline).
//
// Blocked right-looking algorithm on 128-wide panels over the tile-packed
// layout.  For panel kk of every matrix in the batch:
//   1. the diagonal tile is factored in registers and the inverse of its
//      factor written to a scratch tile (diag_factor_tile);
//   2. k_potrf_panel  forms the tiles below it as A_{I,kk} L_kk^{-T}
//                     (an FP64 MFMA product with the inverse);
//   3. k_potrf_update subtracts L_{I,kk} L_{J,kk}^T from the trailing tiles
//                     (FP64 MFMA, the bulk of the flops).
// Step 1 runs as its own launch (k_potrf_diag) for the first panel (and on
// the mixed-precision path for the first panel of each group, or for all
// panels of a large batch); otherwise the update launch that gives the
// diagonal tile its last update goes on to factor it, in the workgroups
// that updated it.
// One launch of each kernel covers the whole batch, so a batch of B
// matrices of order d fills the GPU with B * (trailing tiles) workgroups.
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

// Factor f's source tile at packed offset off, and its shift.
__device__ inline const double* src_tile(const ShiftSrc& src, int64_t S,
                                         int64_t f, int64_t off) {
  return src.H + (f / src.nshift) * S + off;
}
__device__ inline double src_shift(const ShiftSrc& src, int64_t f) {
  const int64_t m = f / src.nshift;
  return src.lam[(m / src.lam_group) * src.nshift + f % src.nshift];
}

// Diagonal tile kk of factor f: its Cholesky factor, held in registers.
// Thread (ti, tk) = (tid % 16, tid / 16) owns the entries (ti + 16a,
// tk + 16b), a >= b, of the tile (x): a two-dimensional cyclic layout, so
// every thread keeps work until the last columns.  Column j is factored
// right-looking (pivot by a refined reciprocal square root, column scaled,
// rank-1 update of the trailing entries).  Each column is published in LDS
// with zeros at rows <= j, so every thread updates whole 16-entry blocks
// without masks.  The step that consumes column j also produces column j+1
// (its block column is updated first, then its 16 owners factor it), so
// one barrier per column suffices; column buffers rotate over three slots.
template <int JB, bool LAST>
__device__ __forceinline__ void diag_step(int jj, double (&x)[8][8],
                                          double* cbuf, int* fail, int ti,
                                          int tk) {
  constexpr int NB1 = LAST ? JB + 1 : JB;  // block column of column j+1
  constexpr bool NEXT = !(LAST && JB == 7);
  const int j = 16 * JB + jj;
  const double* cb = cbuf + (j % 3) * NB;
  double cr[8], cc[8];  // column j at the thread's rows and columns
#pragma unroll
  for (int a = JB; a < 8; ++a) cr[a] = cb[ti + 16 * a];
#pragma unroll
  for (int b = JB; b < 8; ++b) cc[b] = cb[tk + 16 * b];
  double v[8];
  double piv = 0.0;
  const int jn = j + 1, jn16 = jn & 15;
  if constexpr (NEXT) {
#pragma unroll
    for (int a = NB1; a < 8; ++a) x[a][NB1] -= cr[a] * cc[NB1];
    // pivot L(j+1, j+1)^2 sits with thread (jn16, jn16)
    piv = bcast_lane(x[NB1][NB1], 16 * (jn16 & 3) + jn16);
    double ljj, inv;
    sqrt_rsqrt(piv, ljj, inv);
    const bool own = tk == jn16;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      v[a] = 0.0;
      if (a >= NB1) {
        const int i = ti + 16 * a;
        const double sc = x[a][NB1] * inv;
        if (i > jn) v[a] = sc;
        const double nv = i > jn ? sc : (i == jn ? ljj : x[a][NB1]);
        x[a][NB1] = own ? nv : x[a][NB1];
      }
    }
  }
  // the rest of the rank-1 update with column j (block column JB, when it
  // is not NB1, only holds columns <= j: nothing to do)
#pragma unroll
  for (int b = NB1 + 1; b < 8; ++b)
#pragma unroll
    for (int a = b; a < 8; ++a) x[a][b] -= cr[a] * cc[b];
  if (NEXT && tk == jn16) {
    double* cn = cbuf + (jn % 3) * NB;
#pragma unroll
    for (int a = 0; a < 8; ++a) cn[ti + 16 * a] = v[a];
    if (ti == 0 && !(piv > 0.0)) atomicMin(fail, jn);
  }
  __syncthreads();
}

template <int JB>
__device__ __forceinline__ void diag_block(double (&x)[8][8], double* cbuf,
                                           int* fail, int ti, int tk) {
#pragma unroll 1
  for (int jj = 0; jj < 15; ++jj)
    diag_step<JB, false>(jj, x, cbuf, fail, ti, tk);
  diag_step<JB, true>(15, x, cbuf, fail, ti, tk);
}

// Factors one diagonal tile with the whole 256-thread workgroup.  Writes the
// factor (zeros above the diagonal) to `tile` and its inverse (zeros above
// the diagonal) to `li`; the tile's current lower triangle is read from `in`
// (the tile itself, or with SRC the source matrix, plus `shift` on the
// diagonal).  The factor is formed in registers (diag_step), then staged in
// LDS and inverted there by tri_inv_lds (16 x 16 diagonal blocks by forward
// substitution, joined on FP64 MFMA); the column buffers of the first part
// share that LDS.  *info_f gets the global index + 1 of the first
// non-positive pivot when it is the matrix's first failure; with SRC (the
// first panel) it is written either way (0 when no pivot failed).
template <bool SRC>
__device__ __forceinline__ void diag_factor_tile(int64_t d, int kk,
                                                 double* tile, const double* in,
                                                 double shift, int* info_f,
                                                 double* li) {
  __shared__ double S[TRI_LDS];
  __shared__ int fail;
  double* cbuf = S;  // 3 * 128 doubles, free again once the factor is done
  const int tid = threadIdx.x, ti = tid & 15, tk = tid >> 4;
  double x[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      // entries above the diagonal are never used: not read
      x[a][b] = (a > b || ti >= tk) ? in[(tk + 16 * b) * NB + ti + 16 * a] : 0.0;
      if (SRC && a == b && ti == tk && (int64_t)kk * NB + ti + 16 * a < d)
        x[a][b] += shift;
    }
  }
  {  // column 0, by its owners (wave 0)
    const double piv = bcast_lane(x[0][0], 0);
    double ljj, inv;
    sqrt_rsqrt(piv, ljj, inv);
    if (tk == 0) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int i = ti + 16 * a;
        double v = 0.0;
        if (i > 0) {
          x[a][0] *= inv;
          v = x[a][0];
        } else {
          x[a][0] = ljj;
        }
        cbuf[i] = v;
      }
      if (ti == 0) fail = (piv > 0.0) ? NB : 0;
    }
  }
  __syncthreads();
  diag_block<0>(x, cbuf, &fail, ti, tk);
  diag_block<1>(x, cbuf, &fail, ti, tk);
  diag_block<2>(x, cbuf, &fail, ti, tk);
  diag_block<3>(x, cbuf, &fail, ti, tk);
  diag_block<4>(x, cbuf, &fail, ti, tk);
  diag_block<5>(x, cbuf, &fail, ti, tk);
  diag_block<6>(x, cbuf, &fail, ti, tk);
  diag_block<7>(x, cbuf, &fail, ti, tk);
  // the last step ended with a barrier: the column buffers are free
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = ti + 16 * a, k = tk + 16 * b;
      const bool low = a > b || (a == b && ti >= tk);
      const double xv = (a >= b && low) ? x[a][b] : 0.0;
      tile[k * NB + i] = xv;
      if (a >= b) S[blk_off(a, b) + tk * TLD + ti] = xv;
    }
  __syncthreads();
  tri_inv_lds(S);
  // thread (r, h) writes row r of the inverse at the columns 2k + h
  const int r = tid & (NB - 1), h = tid >> 7;
#pragma unroll 8
  for (int k = 0; k < 64; ++k) {
    const int c = 2 * k + h;
    li[c * NB + r] = (r >> 4) < (c >> 4)
                         ? 0.0
                         : S[blk_off(r >> 4, c >> 4) + (c & 15) * TLD + (r & 15)];
  }
  if (tid == 0) {
    const bool bad = fail < NB && (int64_t)kk * NB + fail < d;
    if (SRC)
      *info_f = bad ? kk * NB + fail + 1 : 0;
    else if (bad && *info_f == 0)
      *info_f = kk * NB + fail + 1;
  }
}

// Diagonal tile kk of every matrix of the batch (one workgroup each): the
// factor in place, its inverse at linv + f * lstride + loff.  With SRC (first
// panel only) the tile comes from the source matrix plus its shift.
template <bool SRC>
__global__ void __launch_bounds__(256) k_potrf_diag(int64_t d, int64_t S,
                                                    int kk, double* L,
                                                    int* info, double* linv,
                                                    int64_t lstride,
                                                    int64_t loff,
                                                    ShiftSrc src) {
  const int f = blockIdx.x;
  double* tile = L + (int64_t)f * S + tile_off(kk, kk);
  const double* in = SRC ? src_tile(src, S, f, tile_off(kk, kk)) : tile;
  const double shift = SRC ? src_shift(src, f) : 0.0;
  diag_factor_tile<SRC>(d, kk, tile, in, shift, info + f,
                        linv + (int64_t)f * lstride + loff);
}

// Products of the panel kernel for k in [kb, ke): the wave's 16-row blocks
// j = J0..3 of Linv (rows no[j] .. no[j]+15), each against the wave's
// 64 columns of A^T.  Lane l supplies Linv(no[j] + l%16, k + l/16) and
// A^T(k + l/16, 4(l%16) + bj), so element v of c[j][bj] is
// D'(no[j] + 4v + l/16, 4(l%16) + bj).
template <int J0>
__device__ __forceinline__ void panel_seg(v4d (&c)[4][4], const double* pa,
                                          const int (&no)[4], const double* pb,
                                          int kb, int ke) {
  // operands of the next k step are loaded before this step's products
  v4d bv = ld4(pb + (int64_t)kb * NB);
  double av[4];
#pragma unroll
  for (int j = J0; j < 4; ++j) av[j] = pa[(int64_t)kb * NB + no[j]];
  for (int k0 = kb + 4; k0 <= ke; k0 += 4) {
    v4d bn = bv;
    double an[4];
    if (k0 < ke) {
      bn = ld4(pb + (int64_t)k0 * NB);
#pragma unroll
      for (int j = J0; j < 4; ++j) an[j] = pa[(int64_t)k0 * NB + no[j]];
    }
#pragma unroll
    for (int j = J0; j < 4; ++j)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        c[j][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], bv[bj], c[j][bj],
                                                        0, 0, 0);
    bv = bn;
#pragma unroll
    for (int j = J0; j < 4; ++j) av[j] = an[j];
  }
}

// Panel tile (I, kk), I > kk: X = A L_kk^{-T}, in place (with SRC, A is
// read from the source matrix).  The waves compute
// D'(n,m) = sum_p Linv(n,p) A(m,p) = X(m,n), stored at n*128 + m.  Linv is
// lower triangular, so rows n of the 16-row block b need p < 16(b+1) only.
// Wave w takes the columns m of half w & 1 and four row blocks chosen so
// that both wave pairs do the same work: blocks 0, 1, 6, 7 or 2, 3, 4, 5
// (288 of the 128 k values summed per block column either way, against 512
// for the last 64 rows taken together).  Each block's sum runs only over
// its nonzero k, in segments where the set of active blocks is fixed.
template <bool SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_potrf_panel(int64_t S, int kk, double* L, const double* linv,
              int64_t lstride, int64_t loff, ShiftSrc src) {
  const int f = blockIdx.y;
  const int I = kk + 1 + blockIdx.x;
  const int w = threadIdx.x >> 6, wp = w >> 1, wj = w & 1;
  const int l = threadIdx.x & 63, lq = l >> 4, lr = l & 15;
  double* tile = L + (int64_t)f * S + tile_off(I, kk);
  const double* in = SRC ? src_tile(src, S, f, tile_off(I, kk)) : tile;
  const double* li = linv + (int64_t)f * lstride + loff;
  const double* pa = li + (int64_t)lq * NB + lr;
  const double* pb = in + (int64_t)lq * NB + wj * 64 + 4 * lr;
  v4d c[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) c[j][bj] = v4d{0.0, 0.0, 0.0, 0.0};
  int no[4];
  if (wp == 0) {
    no[0] = 0; no[1] = 16; no[2] = 96; no[3] = 112;
    panel_seg<0>(c, pa, no, pb, 0, 16);
    panel_seg<1>(c, pa, no, pb, 16, 32);
    panel_seg<2>(c, pa, no, pb, 32, 112);
    panel_seg<3>(c, pa, no, pb, 112, 128);
  } else {
    no[0] = 32; no[1] = 48; no[2] = 64; no[3] = 80;
    panel_seg<0>(c, pa, no, pb, 0, 48);
    panel_seg<1>(c, pa, no, pb, 48, 64);
    panel_seg<2>(c, pa, no, pb, 64, 80);
    panel_seg<3>(c, pa, no, pb, 80, 96);
  }
  __syncthreads();  // the whole tile is read before any part is overwritten
  const int m0 = wj * 64 + 4 * lr;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = no[j] + 4 * v + lq;
      st4(tile + n * NB + m0,
          v4d{c[j][0][v], c[j][1][v], c[j][2][v], c[j][3][v]});
    }
}

// acc += sum over the panels c in [c0, c1) of L_Jc(wave rows, :) L_Ic(wave
// columns, :)^T: one stream of 4-long k steps, whose operands are loaded
// two steps ahead of the products, across the panel boundaries too.
__device__ inline void mma_group(Acc64& acc, const double* Lf, int I, int J,
                                 int c0, int c1, int wi, int wj) {
  const int l = threadIdx.x & 63;
  const int64_t lo = (int64_t)(l >> 4) * NB + 4 * (l & 15);
  const int64_t st = 4 * NB;
  const double* pa = Lf + tile_off(J, c0) + wi * 64 + lo;
  const double* pb = Lf + tile_off(I, c0) + wj * 64 + lo;
  v4d a0 = ld4(pa), b0 = ld4(pb), a1 = ld4(pa + st), b1 = ld4(pb + st);
  v4d a2 = ld4(pa + 2 * st), b2 = ld4(pb + 2 * st);
  for (int c = c0; c < c1; ++c) {
    const bool more = c + 1 < c1;
    const double* na = more ? Lf + tile_off(J, c + 1) + wi * 64 + lo : pa;
    const double* nb = more ? Lf + tile_off(I, c + 1) + wj * 64 + lo : pb;
#pragma unroll
    for (int k = 3; k < 35; ++k) {
      const double* qa = k < 32 ? pa + k * st : na + (k - 32) * st;
      const double* qb = k < 32 ? pb + k * st : nb + (k - 32) * st;
      const v4d a3 = ld4(qa), b3 = ld4(qb);
      acc.mma(a0, b0);
      a0 = a1;
      b0 = b1;
      a1 = a2;
      b1 = b2;
      a2 = a3;
      b2 = b3;
    }
    pa = na;
    pb = nb;
  }
}
__device__ inline void mma_group(Acc64F& acc, const double* Lf, int I, int J,
                                 int c0, int c1, int wi, int wj) {
  for (int c = c0; c < c1; ++c)
    mma_panel_f32(acc, Lf + tile_off(J, c) + wi * 64, NB,
                  Lf + tile_off(I, c) + wj * 64, NB, NB);
}

// Where a fused diagonal factorization writes: the inverse of tile j0 of
// factor f goes to linv + f * lstride + loff, a failed pivot to info[f].
// dc0 >= 0: tile (j0, j0) already holds the panels before dc0 (a previous
// launch took them ahead), so this launch sums only [dc0, c1) for it.
// pre: the launch also takes the panels [c0, c1) into tile (j0+1, j0+1)
// ahead of its own column update.
struct DiagOut {
  int* info;
  double* linv;
  int64_t lstride;
  int64_t loff;
  int fuse;  // 1: the launch also factors diagonal tile (j0, j0)
  int dc0;
  int pre;
};

// Trailing tile (I,J): A_IJ -= sum_{c in [c0,c1)} L_Ic L_Jc^T, for the
// tiles of the triangle j0 <= J <= I (mode 0) or of the `mode` whole
// columns J = j0 .. j0+mode-1 (mode > 0).
// The wave computes D'(n,m) = sum_p L_Jc(n,p) L_Ic(m,p) = update(m,n) and
// subtracts it from the tile in its epilogue.  Two workgroups share a CU
// (the register budget is capped for two waves per SIMD), so one's
// read-modify-write epilogue overlaps the other's products.  Logical
// workgroup ids are laid out matrix by matrix and spread over the XCDs in
// contiguous ranges.
// In both modes tile (j0, j0) receives its last update in this launch.  With
// dout.fuse (FUSABLE instantiations, whose register budget leaves room for
// it) the first nfac workgroups take those tiles, one per matrix, and after
// the update go on to factor it (diag_factor_tile), so
// the diagonal factorization runs while the rest of the launch is still
// updating; the other workgroups take the remaining tiles.  With dout.pre
// the last nfac workgroups update tile (j0+1, j0+1) ahead (see DiagOut), so
// the next column's diagonal workgroup starts its factorization sooner.
template <typename ACC, bool SRC, bool FUSABLE>
__device__ inline void potrf_update_body(int64_t S, int nt, int j0, int mode,
                                         int c0, int c1, int ntile, double* L,
                                         int64_t d, const ShiftSrc& src,
                                         const DiagOut& dout) {
  const bool fuse = FUSABLE && dout.fuse;
  const int nfac = (int)gridDim.x / (ntile + dout.pre);
  const int nmain = nfac * ntile;  // workgroups of the launch's own tiles
  int f, t;
  const bool ahead = (int)blockIdx.x >= nmain;
  if (ahead) {
    f = (int)blockIdx.x - nmain;
    t = -1;
  } else if (fuse) {
    if ((int)blockIdx.x < nfac) {
      f = blockIdx.x;
      t = 0;
    } else {
      const int rest = ntile - 1;  // >= 1 here: the grid holds more tiles
      const int id = xcd_remap((int)blockIdx.x - nfac, nmain - nfac);
      f = id / rest;
      t = 1 + (id - f * rest);
    }
  } else {
    const int id = xcd_remap(blockIdx.x, nmain);
    f = id / ntile;
    t = id - f * ntile;
  }
  // tile (j0, j0) taken over from a launch that started its sum
  const bool resumed = t == 0 && dout.dc0 >= 0;
  const int ca = resumed ? dout.dc0 : c0;
  // with SRC the tile is read from the source matrix, unless an earlier
  // launch has touched it already
  const bool from_src = SRC && !resumed;
  int I, J;
  if (ahead) {
    I = J = j0 + 1;
  } else if (mode == 0) {
    const int r = tri_row(t);
    I = j0 + r;
    J = j0 + (t - (int)tri(r));
  } else {
    // `mode` whole columns j0, j0+1, ..., enumerated column by column
    int J0 = j0, tt = t;
    while (tt >= nt - J0) {
      tt -= nt - J0;
      ++J0;
    }
    I = J0 + tt;
    J = J0;
  }
  const int w = threadIdx.x >> 6, wi = w >> 1, wj = w & 1;
  double* Lf = L + (int64_t)f * S;
  double* ct = Lf + tile_off(I, J);
  if (!(I == J && wi > wj)) {  // that block lies strictly above the diagonal
    // the tile's current value: L itself, or (first touch) the source matrix
    const double* cs = from_src ? src_tile(src, S, f, tile_off(I, J)) : ct;
    const LaneXY lx;
    const int m0 = wj * 64 + lx.col0();
    ACC acc;
    acc.zero();
    mma_group(acc, Lf, I, J, ca, c1, wi, wj);
    const double shift = (from_src && I == J) ? src_shift(src, f) : 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) {
        const int n = wi * 64 + ACC::row_of(lx.lq, v, bi);
        double* p = ct + n * NB + m0;
        const double* q = cs + n * NB + m0;
        const v4d val = acc.row(v, bi);
        if (I != J || wi != wj) {
          st4(p, ld4(q) - val);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (m0 + e >= n) {
              double cv = q[e];
              if (from_src && m0 + e == n && (int64_t)I * NB + n < d) cv += shift;
              p[e] = cv - val[e];
            }
        }
      }
  }
  if constexpr (FUSABLE) {
    if (fuse && t == 0) {
      // the tile's lower triangle, just stored by three of the four waves,
      // is read back by the whole workgroup once the barrier has passed
      __syncthreads();
      diag_factor_tile<false>(d, j0, ct, ct, 0.0, dout.info + f,
                              dout.linv + (int64_t)f * dout.lstride + dout.loff);
    }
  }
}

template <bool SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_potrf_update(int64_t S, int nt, int j0, int mode, int c0, int c1, int ntile,
               double* L, int64_t d, ShiftSrc src, DiagOut dout) {
  potrf_update_body<Acc64, SRC, true>(S, nt, j0, mode, c0, c1, ntile, L, d,
                                      src, dout);
}

// Mixed precision: the same update with the products on FP32 MFMA (operands
// rounded to FP32, FP32 accumulation over the 256-long sums); the tile
// itself stays FP64.  FP32 accumulators take half the registers, so four
// workgroups share a CU (measured faster than two at d = 4096); that budget
// leaves no room for the diagonal factorization.  The trailing updates use
// this form, and the first panel of each group has its own diagonal launch.
template <bool SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_potrf_update_f32(int64_t S, int nt, int j0, int mode, int c0, int c1,
                   int ntile, double* L, int64_t d, ShiftSrc src, int dc0,
                   int pre) {
  potrf_update_body<Acc64F, SRC, false>(
      S, nt, j0, mode, c0, c1, ntile, L, d, src,
      DiagOut{nullptr, nullptr, 0, 0, 0, dc0, pre});
}

// The mixed-precision column updates inside a group (short launches, with
// the diagonal factorization on the critical path) at two workgroups per CU,
// which leaves room for factoring the diagonal tile the launch completes.
template <bool SRC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_potrf_update_f32_diag(int64_t S, int nt, int j0, int mode, int c0, int c1,
                        int ntile, double* L, int64_t d, ShiftSrc src,
                        DiagOut dout) {
  potrf_update_body<Acc64F, SRC, true>(S, nt, j0, mode, c0, c1, ntile, L, d,
                                       src, dout);
}

// Side stream for look-ahead: created once per device on first use, with
// the default priority, and a small ring of events.
struct SideStream {
  bool ready = false;
  hipStream_t stream = nullptr;
  hipEvent_t ev[8] = {};
};
static std::mutex g_side_mu;
static SideStream g_side[64];

static SideStream* side_stream() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  SideStream& ss = g_side[dev];
  if (!ss.ready) {
    if (hipStreamCreateWithFlags(&ss.stream, hipStreamNonBlocking) != hipSuccess)
      return nullptr;
    for (hipEvent_t& e : ss.ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return nullptr;
    ss.ready = true;
  }
  return &ss;
}

// Panels in groups of G with a delayed update: before its diagonal
// factorization, column kk+u receives the group's earlier panels (K = 128 u);
// after the group, one update of rank 128 G reaches the rest of the trailing
// matrix.  On the FP64 path each of these launches also factors the
// diagonal tile it completes (tile kk+u, or the next group's first).  With
// the look-ahead option on, that update is split: the G columns the next
// group factors stay on the caller's stream, the remainder
// runs on a side stream, so the next group's diagonal factorizations, panel
// solves and column updates (short, latency-bound launches) overlap the bulk
// of the update.  The side update is joined before the next group's own
// trailing update, the first launch that touches the same tiles.
hipError_t launch_potrf_blocked(int64_t d, int nfac, const ShiftSrc& src,
                                double* L, int* info, double* linv_ws,
                                int keep_linv, int mixed, int lookahead,
                                int group, hipStream_t s,
                                const PanelHook* hook) {
  const int nt = (int)ntiles_of(d);
  const int64_t S = packed_elems_of(d);
  // inverse of panel kk of factor f: at f * NB2 (scratch, overwritten by
  // the next panel) or, kept for the solves, at (f * nt + kk) * NB2
  const int64_t lstride = keep_linv ? (int64_t)nt * NB2 : NB2;
  const bool has_src = src.H != nullptr;
  std::unique_lock<std::mutex> lk(g_side_mu, std::defer_lock);
  if (lookahead) lk.lock();
  SideStream* side = lookahead ? side_stream() : nullptr;
  // Every diagonal tile but the first is factored by the update launch that
  // completes it: the column update inside a group, or (FP64 path) the
  // trailing update after it.  The mixed path launches k_potrf_diag itself
  // for the first panel of each group, and for every panel when the batch
  // is large: its fused column updates run two workgroups per CU instead of
  // four, which costs more than the fusion saves once the launches fill the
  // GPU (measured at d = 4096: 30 matrices 0.35 ms faster, 320 matrices
  // 0.5 ms slower).
  const bool fuse_cols = !mixed || nfac < 128;
  const bool fuse_trail = !mixed;
  auto diag_panel = [&](int kk, bool first, bool factored) {
    const int64_t loff = keep_linv ? (int64_t)kk * NB2 : 0;
    if (!factored && first)
      PICHOL_LAUNCH(k_potrf_diag<true>, dim3((unsigned)nfac), dim3(256), 0, s,
                    d, S, kk, L, info, linv_ws, lstride, loff, src);
    else if (!factored)
      PICHOL_LAUNCH(k_potrf_diag<false>, dim3((unsigned)nfac), dim3(256), 0, s,
                    d, S, kk, L, info, linv_ws, lstride, loff, src);
    const int rest = nt - kk - 1;
    if (rest <= 0) return;
    const dim3 grid((unsigned)rest, (unsigned)nfac);
    if (first)
      PICHOL_LAUNCH(k_potrf_panel<true>, grid, dim3(256), 0, s, S, kk, L,
                    linv_ws, lstride, loff, src);
    else
      PICHOL_LAUNCH(k_potrf_panel<false>, grid, dim3(256), 0, s, S, kk, L,
                    linv_ws, lstride, loff, src);
  };
  // fd: this launch also factors diagonal tile (j0, j0); dc0, pre: see
  // DiagOut
  auto update = [&](hipStream_t st, int j0, int mode, int c0, int c1,
                    bool first, bool fd, int dc0 = -1, bool pre = false) {
    const int rest = nt - j0;
    if (rest <= 0) return;
    const int m = mode == 0 ? 0 : (mode < rest ? mode : rest);
    const int ntile = m == 0 ? (int)tri(rest) : m * rest - m * (m - 1) / 2;
    const int npre = pre ? 1 : 0;
    const dim3 grid((unsigned)((ntile + npre) * nfac));
    const DiagOut dout{info, linv_ws, lstride,
                       keep_linv ? (int64_t)j0 * NB2 : 0, fd ? 1 : 0, dc0,
                       npre};
    if (mixed && fd && first)
      PICHOL_LAUNCH(k_potrf_update_f32_diag<true>, grid, dim3(256), 0, st, S,
                    nt, j0, m, c0, c1, ntile, L, d, src, dout);
    else if (mixed && fd)
      PICHOL_LAUNCH(k_potrf_update_f32_diag<false>, grid, dim3(256), 0, st, S,
                    nt, j0, m, c0, c1, ntile, L, d, src, dout);
    else if (mixed && first)
      PICHOL_LAUNCH(k_potrf_update_f32<true>, grid, dim3(256), 0, st, S, nt,
                    j0, m, c0, c1, ntile, L, d, src, dc0, npre);
    else if (mixed)
      PICHOL_LAUNCH(k_potrf_update_f32<false>, grid, dim3(256), 0, st, S, nt,
                    j0, m, c0, c1, ntile, L, d, src, dc0, npre);
    else if (first)
      PICHOL_LAUNCH(k_potrf_update<true>, grid, dim3(256), 0, st, S, nt, j0, m,
                    c0, c1, ntile, L, d, src, dout);
    else
      PICHOL_LAUNCH(k_potrf_update<false>, grid, dim3(256), 0, st, S, nt, j0,
                    m, c0, c1, ntile, L, d, src, dout);
  };
  const int G = group > 0 ? group : option_panel_group();
  int ring = 0;
  bool pending = false;  // a side-stream update not yet joined
  hipEvent_t joined = nullptr;
  for (int kk = 0; kk < nt; kk += G) {
    // the first group's launches are the first to touch every tile
    const bool first = has_src && kk == 0;
    for (int u = 0; u < G && kk + u < nt; ++u) {
      // column kk+u's launch also takes the group's panels so far into
      // diagonal tile kk+u+1, whose own launch then sums only the newest
      // panel before that tile's factorization starts (the same sums on
      // every path, so results do not depend on the batch size)
      if (u > 0)
        update(s, kk + u, 1, kk, kk + u, first, fuse_cols,
               u >= 2 ? kk + u - 1 : -1, u + 1 < G && kk + u + 1 < nt);
      // tile kk (u = 0) was factored by the previous group's trailing update
      // on the FP64 path
      diag_panel(kk + u, first && u == 0,
                 u > 0 ? fuse_cols : (fuse_trail && kk > 0));
      if (hook && kk + u == hook->col) {
        const hipError_t e = hook->fn(hook->ctx);
        if (e != hipSuccess) return e;
      }
    }
    if (kk + G >= nt) break;
    if (pending) {
      pending = false;
      const hipError_t e = hipStreamWaitEvent(s, joined, 0);
      if (e != hipSuccess) return e;
    }
    if (side && kk + 2 * G < nt) {
      hipEvent_t ready = side->ev[ring++ & 7];
      hipError_t e = hipEventRecord(ready, s);
      if (e != hipSuccess) return e;
      update(s, kk + G, G, kk, kk + G, first, fuse_trail);  // the next group's columns
      e = hipStreamWaitEvent(side->stream, ready, 0);
      if (e != hipSuccess) return e;
      update(side->stream, kk + 2 * G, 0, kk, kk + G, first, false);
      joined = side->ev[ring++ & 7];
      e = hipEventRecord(joined, side->stream);
      if (e != hipSuccess) {
        // the side work is enqueued; make the caller's stream wait for all
        // of the side stream's work before reporting
        (void)hipStreamSynchronize(side->stream);
        return e;
      }
      pending = true;
    } else {
      update(s, kk + G, 0, kk, kk + G, first, fuse_trail);
    }
  }
  if (pending) {
    const hipError_t e = hipStreamWaitEvent(s, joined, 0);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace pichol
