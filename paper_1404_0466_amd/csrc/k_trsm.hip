// Forward and back substitution (Sec. 3.2) for many right-hand sides and
// many factors at once, blocked over 128-row tiles.
//
// The right-hand sides of one fold live in a row-major slab Z (dp x ldz);
// columns t*c .. t*c+c-1 belong to lambda index t.  Forward substitution
// walks the tile rows i = 0..nt-1: solve the diagonal block of every
// lambda, then subtract the contribution of the solved rows from every
// later tile row (update kernels).  Back substitution walks the tile rows
// in reverse with the transposed blocks.
//
// The diagonal steps multiply by stored inverses of the diagonal blocks
// (k_diag_apply), out of place between Z and a second slab X, so several
// workgroups can share one (fold, lambda).  Interpolated factors (Sec. 3.3)
// are never materialised: their diagonal blocks are evaluated and inverted
// once, up front, all in parallel (k_diag_inv), and the off-diagonal update
// of all lambdas is one FP64 MFMA product
// Lhat_t(I,i) U_t = sum_p Theta_p(I,i) (tau_t^p U_t), so each coefficient
// tile is read once per step for all q values.  Exact factors (the
// per-lambda baseline) use one factor per lambda and the inverses their
// factorization kept; factors given without inverses are solved in place by
// substitution (k_diag_solve).
#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

// Z[m][i][col] = B[m][i][col % c] for col < q*c, 0 beyond; flags cleared.
__global__ void __launch_bounds__(256) k_slab_init(int64_t dp, int q, int c,
                                                   int64_t ldz,
                                                   const double* B, double* Z,
                                                   int* flags) {
  const int64_t m = blockIdx.y;
  const int64_t n = dp * ldz;
  const int64_t qc = (int64_t)q * c;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ldz, col = e % ldz;
    Z[m * n + e] = col < qc ? B[(m * dp + i) * c + col % c] : 0.0;
  }
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t < q; t += blockDim.x) flags[m * q + t] = 0;
}

// Where the factors come from.
struct FactorSrc {
  const double* base;
  int64_t S;      // packed elements per triangle
  int M;          // interpolated: coefficient planes per fold
  int exact;      // 1: factor (m,t) at base + (m*nper + t)*S
  int nper;       // lambda values per fold
  const double* tau;  // interpolated: tau_t = lambda_t / lambda_ref
};

// Solve the diagonal block of tile row i for lambda t = blockIdx.x of fold
// m = blockIdx.y, in place in the slab: forward L x = z, or back L^T x = z.
template <bool FWD>
__global__ void __launch_bounds__(256) k_diag_solve(int64_t d, int i,
                                                    FactorSrc src, int c,
                                                    int64_t ldz, double* Z,
                                                    int* flags) {
  __shared__ double a[NB * LDS_LD];
  const int t = blockIdx.x;
  const int64_t m = blockIdx.y;
  const int tid = threadIdx.x;
  const int64_t dp = ntiles_of(d) * NB;
  const int64_t toff = tile_off(i, i);
  {
    const double* p = src.exact ? src.base + (m * src.nper + t) * src.S + toff
                                : src.base + m * src.M * src.S + toff;
    const int M = src.exact ? 1 : src.M;
    const double tv = src.exact ? 1.0 : src.tau[t];
#pragma unroll
    for (int it = 0; it < 16; it += 8) {
      v4d acc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
      double pw = 1.0;
      for (int q = 0; q < M; ++q) {
        v4d v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = ld4(p + q * src.S + ((it + u) * 256 + tid) * 4);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += pw * v[u];
        pw *= tv;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = ((it + u) * 256 + tid) * 4;
#pragma unroll
        for (int x = 0; x < 4; ++x)
          a[(e >> 7) * LDS_LD + ((e + x) & (NB - 1))] = acc[u][x];
      }
    }
  }
  __syncthreads();
  if (FWD && tid < NB && (int64_t)i * NB + tid < d &&
      !(a[tid * LDS_LD + tid] > 0.0))
    atomicOr(flags + m * src.nper + t, 2);

  const int lane = tid & 63, w = tid >> 6;
  const int r0 = lane, r1 = lane + 64;
  double* zbase = Z + (m * dp + (int64_t)i * NB) * ldz + (int64_t)t * c;
  for (int cg = 0; cg < c; cg += 16) {
    double z[4][2];
    int ncol = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cc = cg + w + 4 * u;
      if (cc < c && cc < cg + 16) {
        z[u][0] = zbase[(int64_t)r0 * ldz + cc];
        z[u][1] = zbase[(int64_t)r1 * ldz + cc];
        ncol = u + 1;
      } else {
        z[u][0] = z[u][1] = 0.0;
      }
    }
    if (FWD) {
      for (int j = 0; j < NB; ++j) {
        const double piv = a[j * LDS_LD + j];
        const double l0 = a[j * LDS_LD + r0], l1 = a[j * LDS_LD + r1];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (u >= ncol) break;
          const double xj = bcast_lane(j < 64 ? z[u][0] : z[u][1], j & 63) / piv;
          if (r0 == j) z[u][0] = xj; else if (r0 > j) z[u][0] -= l0 * xj;
          if (r1 == j) z[u][1] = xj; else if (r1 > j) z[u][1] -= l1 * xj;
        }
      }
    } else {
      for (int j = NB - 1; j >= 0; --j) {
        const double piv = a[j * LDS_LD + j];
        // L(j, r) is row j, column r of the tile
        const double l0 = a[r0 * LDS_LD + j], l1 = a[r1 * LDS_LD + j];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (u >= ncol) break;
          const double xj = bcast_lane(j < 64 ? z[u][0] : z[u][1], j & 63) / piv;
          if (r0 == j) z[u][0] = xj; else if (r0 < j) z[u][0] -= l0 * xj;
          if (r1 == j) z[u][1] = xj; else if (r1 < j) z[u][1] -= l1 * xj;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cc = cg + w + 4 * u;
      if (u < ncol) {
        zbase[(int64_t)r0 * ldz + cc] = z[u][0];
        zbase[(int64_t)r1 * ldz + cc] = z[u][1];
      }
    }
  }
}

// Inverse of diagonal block i of the interpolated factor for lambda t of
// fold m.  The block is evaluated from the coefficient planes into LDS
// (sum_p tau^p Theta_p, p increasing; entries above the diagonal are not
// read), then inverted in place by tri_inv_lds (16 x 16 diagonal blocks by
// forward substitution, joined on FP64 MFMA).  77 KB of LDS, so two
// workgroups share a CU.  Writes the inverse, column-major with zeros above
// the diagonal, to dinv.  A non-positive diagonal entry of the block sets
// flag bit1.  The grid covers the tile rows i0, i0+1, ...
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_diag_inv(int64_t d, FactorSrc src, double* dinv, int* flags, int i0) {
  __shared__ double S[TRI_LDS];
  const int i = i0 + (int)blockIdx.x, t = blockIdx.y;
  const int64_t m = blockIdx.z;
  const int nt = (int)ntiles_of(d);
  const int tid = threadIdx.x;
  const double* planes = src.base + m * src.M * src.S + tile_off(i, i);
  const double tau = src.tau[t];
  // thread (r, h) = (tid % 128, tid / 128) evaluates row r at the columns
  // c = 2k + h, k = 0..63.  Every load is unconditional (all inside the
  // tile) and entries above the diagonal are dropped by a select, so all of
  // a plane's loads are in flight at once.
  const int r = tid & (NB - 1), h = tid >> 7;
  double x[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) x[k] = 0.0;
  double pw = 1.0;
  for (int p = 0; p < src.M; ++p) {
    const double* pp = planes + p * src.S + r;
    double v[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) v[k] = pp[(2 * k + h) * NB];
#pragma unroll
    for (int k = 0; k < 64; ++k) {
      const double y = x[k] + pw * v[k];
      x[k] = r >= 2 * k + h ? y : 0.0;
    }
    pw *= tau;
  }
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 64; ++k) {
    const int c = 2 * k + h;
    if ((r >> 4) >= (c >> 4))
      S[blk_off(r >> 4, c >> 4) + (c & 15) * TLD + (r & 15)] = x[k];
    if (r == c && (int64_t)i * NB + r < d && !(x[k] > 0.0)) bad = true;
  }
  if (bad) atomicOr(flags + m * src.nper + t, 2);
  __syncthreads();
  tri_inv_lds(S);
  double* out = dinv + ((m * src.nper + t) * nt + i) * (int64_t)NB2;
#pragma unroll 8
  for (int k = 0; k < 64; ++k) {
    const int c = 2 * k + h;
    out[c * NB + r] = (r >> 4) < (c >> 4)
                          ? 0.0
                          : S[blk_off(r >> 4, c >> 4) + (c & 15) * TLD + (r & 15)];
  }
}

// Apply the stored inverse of diagonal block i to the slab rows of tile i,
// out of place: dst rows of tile i = M (src rows of tile i), for the c
// columns of lambda t of fold m.  The inverse is stored column-major
// (entry (r,k) at k*128 + r); forward steps apply it (M lower triangular),
// back steps its transpose (M(r,k) = mat[r*128 + k], upper triangular).  Four workgroups per (fold, lambda) each own 32 rows of the
// result; only the triangle's nonzero columns k of those rows are read
// (k < r0 + 32 forward, k >= r0 backward).  The 32 rows of M and the
// 128-row block of right-hand sides sit in LDS; thread (row, pair) sums two
// columns over k in increasing order.  Grid x = 4 * lambda + quarter; nper
// is the number of lambdas (the slab holds nper * c columns, then zero
// padding up to ldz).
template <bool FWD>
__global__ void __launch_bounds__(256) k_diag_apply(int64_t d, int i, int nper,
                                                    int c, const double* mats,
                                                    int64_t ldz,
                                                    const double* src,
                                                    double* dst) {
  __shared__ v4d ms4[NB * 8];      // ms[k*32 + rr] = M(r0 + rr, k)
  __shared__ double2 zs2[NB * 8];  // zs[k*16 + u] = src(k, cg + u)
  double* ms = reinterpret_cast<double*>(ms4);
  double* zs = reinterpret_cast<double*>(zs2);
  const int qt = blockIdx.x & 3, t = blockIdx.x >> 2;
  const int64_t m = blockIdx.y;
  const int nt = (int)ntiles_of(d);
  const int tid = threadIdx.x, rr = tid & 31, pr = tid >> 5;
  const int r0 = 32 * qt;
  const int klo = FWD ? 0 : r0, khi = FWD ? r0 + 32 : NB;
  const int64_t dp = (int64_t)nt * NB;
  const double* M = mats + ((m * nper + t) * nt + i) * (int64_t)NB2;
  const int64_t zoff = (m * dp + (int64_t)i * NB) * ldz + (int64_t)t * c;
  const double* zs_src = src + zoff;
  double* zd = dst + zoff;
  // The needed part of M in at most four 32-byte pieces per thread, all
  // loaded before any is stored (pieces past the end re-read the last one,
  // inside the tile, and are not stored).
  const int npc = (khi - klo) * 8;  // pieces
  // Right-hand sides of columns cg .. cg+15 (zero past the lambda's c
  // columns): every load unconditional, at most column c-1, so the loads of
  // the first block are in flight together with those of M.
  auto load_z = [&](int cg, double (&zv)[8]) {
    const int cn = (c - cg) < 16 ? (c - cg) : 16;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u, k = e >> 4, cc = e & 15;
      const double x = zs_src[(int64_t)k * ldz + cg + min(cc, cn - 1)];
      zv[u] = cc < cn ? x : 0.0;
    }
  };
  double zv[8];
  load_z(0, zv);
  if (FWD) {
    // rows r0..r0+31 of M over the needed k: eight 32-byte pieces per k
    v4d v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = min(tid + 256 * u, npc - 1);
      const int k = klo + (e >> 3), part = e & 7;
      v[u] = ld4(M + (int64_t)k * NB + r0 + part * 4);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      if (e < npc) *(v4d*)(ms + (klo + (e >> 3)) * 32 + (e & 7) * 4) = v[u];
    }
  } else {
    // M(r0 + rr, k) = mat[(r0 + rr) * 128 + k]: 32-byte pieces along k,
    // consecutive lanes on consecutive rows (conflict-free LDS stores)
    v4d v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = min(tid + 256 * u, npc - 1);
      v[u] = ld4(M + (int64_t)(r0 + (e & 31)) * NB + klo + 4 * (e >> 5));
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      if (e < npc) {
        const int rr = e & 31, k = klo + 4 * (e >> 5);
#pragma unroll
        for (int x = 0; x < 4; ++x) ms[(k + x) * 32 + rr] = v[u][x];
      }
    }
  }
  for (int cg = 0; cg < c; cg += 16) {
    const int cn = (c - cg) < 16 ? (c - cg) : 16;
    if (cg) {
      __syncthreads();
      load_z(cg, zv);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) zs[tid + 256 * u] = zv[u];
    __syncthreads();
    double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
    for (int k = klo; k < khi; ++k) {
      const double mv = ms[k * 32 + rr];
      const double2 zz = *(const double2*)(zs + k * 16 + 2 * pr);
      a0 += mv * zz.x;
      a1 += mv * zz.y;
    }
    double* out = zd + (int64_t)(r0 + rr) * ldz + cg + 2 * pr;
    if (2 * pr < cn) out[0] = a0;
    if (2 * pr + 1 < cn) out[1] = a1;
  }
  // the last lambda's workgroups also keep the slab's padding columns
  // (q*c .. ldz) of their rows at zero in the destination
  if (t == nper - 1) {
    const int64_t qc = (int64_t)nper * c;
    double* pad = dst + (m * dp + (int64_t)i * NB + r0) * ldz;
    for (int64_t e = tid; e < 32 * (ldz - qc); e += 256) {
      const int64_t r = e / (ldz - qc);
      pad[r * ldz + qc + e % (ldz - qc)] = 0.0;
    }
  }
}

// Off-diagonal update for interpolated factors.  Forward step i: rows of
// tile I > i lose sum_p Theta_p(I,i) (tau^p .* U_i); backward step i: rows
// of tile I < i lose sum_p Theta_p(i,I)^T (tau^p .* W_i), read from the
// row-major copy of the planes.  A workgroup owns a 64 x 128 block (half of
// the tile's rows, one 128-column block of the slab); its four waves split
// it into two 64-column halves and the 128-long sums of every plane into two
// 64-long halves, so a launch has twice as many, twice as short workgroups
// (the last round of a launch is less empty).  The first half's
// accumulators start from the slab rows being updated, the second half's
// from zero; the second hands its partial sums over in LDS and the first
// adds them (a fixed order).  Products are subtracted (negative scale).
// Logical workgroup ids run over the column blocks fastest, so the blocks
// that share a coefficient tile meet on one XCD.
template <bool FWD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_update_interp(
    int64_t d, int i, const double* theta, const double* theta_t, int64_t S,
    int M, int q, int c, const double* tau, int64_t ldz, int ncb, int nrows,
    const double* X, double* Z) {
  __shared__ v4d xch[2][16][64];  // partial sums of the k-second-half waves
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int cb = id % ncb;
  const int rest = id / ncb;
  const int rh = rest & 1;  // row half of the tile
  const int row = (rest >> 1) % nrows;
  const int64_t m = (rest >> 1) / nrows;
  const int I = FWD ? i + 1 + row : row;
  const int w = threadIdx.x >> 6, wj = w & 1, kh = w >> 1;
  const int l = threadIdx.x & 63;
  const int64_t dp = ntiles_of(d) * NB;
  const LaneXY lx;
  const int64_t col = (int64_t)cb * NB + wj * 64 + lx.col0();
  const int64_t qc = (int64_t)q * c;
  v4d tau4;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    tau4[e] = (col + e) < qc ? tau[(col + e) / c] : 0.0;

  const double* planes = FWD ? theta + m * M * S + tile_off(I, i)
                             : theta_t + m * M * S + tile_off(i, I);
  const double* bsrc = X + (m * dp + (int64_t)i * NB) * ldz + cb * NB + wj * 64;
  double* zt = Z + (m * dp + (int64_t)I * NB + rh * 64) * ldz + col;
  Acc64 acc;
  if (kh == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
        acc.set_row(v, bi, ld4(zt + (int64_t)lx.row(v, bi) * ldz));
  } else {
    acc.zero();
  }
  v4d scale = {-1.0, -1.0, -1.0, -1.0};
  for (int p = 0; p < M; ++p) {
    mma_panel_scaled(acc, planes + p * S + rh * 64 + (int64_t)kh * 64 * NB, NB,
                     bsrc + (int64_t)kh * 64 * ldz, ldz, 64, scale);
    scale *= tau4;
  }
  if (kh == 1) {
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) xch[wj][bi * 4 + bj][l] = acc.c[bi][bj];
  }
  __syncthreads();
  if (kh == 0) {
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) acc.c[bi][bj] += xch[wj][bi * 4 + bj][l];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
        st4(zt + (int64_t)lx.row(v, bi) * ldz, acc.row(v, bi));
  }
}

// Per-lambda form of one interpolated solve step, with the next diagonal
// solve fused in.  The right-hand sides are taken in units of one lambda
// and up to 16 of its columns (unit u = t * ncu + h, ncu = ceil(c / 16),
// columns t*c + 16h ...).  A workgroup owns the 128 rows of one tile row I
// and U consecutive units; wave w takes the 64 rows of half
// rh = w & 1 and the half kh = w >> 1 of the 128-long sums, for all of the
// workgroup's units.  For every k step it loads the r+1 coefficient tiles'
// values once, evaluates each unit's Lhat_t(I, i) = sum_p tau_t^p
// Theta_p(I, i) from them in registers (Horner's rule), and multiplies that
// with the unit's 16 columns on FP64 MFMA.  Against the stacked product
// (every column scaled by each of the r+1 powers, K = (r+1) * 128) this
// takes (r+1) * c / 16 times fewer products per column when c <= 16, at 2r
// fused multiply-adds per operand value on the vector unit.  The second
// half of the sums is handed to the first through LDS (a fixed order).
// The workgroups of tile row i+1 (forward; i-1 backward) come first in the
// grid.  After their update they stage the updated rows in LDS and multiply
// them by the stored inverse of that diagonal block (backward: by its
// transpose), writing the block the next step reads, so the steps need no
// diagonal launches of their own.  Their updated rows themselves are not
// stored: no later step reads them.
//   forward : dst rows of I > i  -=  Lhat(I, i) src(i);
//             out(i+1) = Linv(i+1) dst(i+1)
//   backward: dst rows of I < i  -=  Lhat(i, I)^T src(i);
//             out(i-1) = Linv(i-1)^T dst(i-1)
// theta is the column-major planes (forward) or their row-major copy
// (backward), so that A(row, k) sits at k * 128 + row either way.  MT is
// the number of planes r+1 (0: any, read inside the k loop).
// U units per workgroup: 4, or 2 for launches too small to fill the GPU
// and for the steps that run alone (half the serial work per workgroup,
// twice the workgroups; 164 registers, so three waves share a SIMD where
// the four-unit form's 242 allow two).
template <bool FWD, int MT, int U>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(U == 2 ? 3 : 2, U == 2 ? 3 : 2)))
k_step_interp(int64_t d, int i, int nmat, const double* theta, int64_t S,
              int M, int q, int c, const double* tau, int64_t ldz, int nrows,
              int ngrp, const double* dinv, const double* src, double* dst,
              double* out) {
  __shared__ double zl[U * NB * 16];  // [unit][row][column]
  const int nt = (int)ntiles_of(d);
  const int64_t dp = (int64_t)nt * NB;
  // the fused tile row's workgroups take the first ids, one per XCD in
  // turn; the others are spread over the XCDs in contiguous ranges, the
  // units of one coefficient tile together
  const int nf = nmat * ngrp;
  int id = blockIdx.x;
  if (id >= nf) id = nf + xcd_remap(id - nf, (int)gridDim.x - nf);
  const int g = id % ngrp;
  const int64_t m = (id / ngrp) % nmat;
  const int ro = id / (ngrp * nmat);
  const int I = FWD ? i + 1 + ro : i - 1 - ro;
  // wave-uniform indices (kept in scalar registers), so that every address
  // below is a uniform base plus a 32-bit lane offset
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int rh = w & 1, kh = w >> 1;
  const int l = threadIdx.x & 63, lq = l >> 4, lr = l & 15;
  const int ncu = (c + 15) >> 4;
  const int nunits = q * ncu;
  const int ldzi = (int)ldz;
  int tt[U];
  unsigned cofs[U];  // slab column of the lane's entry of each unit
  bool ok[U];   // the lane's column belongs to a valid unit
  double tv[U];
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const int u = g * U + j;
    const int uc = u < nunits ? u : nunits - 1;
    const int t = uc / ncu, h = uc - t * ncu;
    const int ncol = (c - 16 * h) < 16 ? (c - 16 * h) : 16;
    tt[j] = t;
    ok[j] = u < nunits && lr < ncol;
    cofs[j] = (unsigned)(t * c + 16 * h + (lr < ncol ? lr : ncol - 1));
    tv[j] = tau[t];
  }
  const int kb = 64 * kh;  // the wave's k range [kb, kb + 64)
  const double* pl = theta + m * M * S + (FWD ? tile_off(I, i) : tile_off(i, I)) +
                     rh * 64 + (int64_t)kb * NB;
  const unsigned plo = (unsigned)(lq * NB + 4 * lr);
  double* drow = dst + (m * dp + (int64_t)I * NB + rh * 64) * ldz;
  unsigned dro[U];
#pragma unroll
  for (int j = 0; j < U; ++j) dro[j] = (unsigned)(4 * lq * ldzi) + cofs[j];
  // the first k half starts from the rows being updated; element v of
  // block bi is row 16v + 4lq + bi of the half, column lr of the unit
  v4d acc[U][4];
  if (kh == 0) {
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double x = *at_elem(drow + (int64_t)(16 * v + bi) * ldz, dro[j]);
          acc[j][bi][v] = ok[j] ? x : 0.0;
        }
  } else {
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) acc[j][bi] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  // (MT > 0) the coefficient values of the first k step, loaded before the
  // staging below so that both round trips to memory overlap
  v4d th[3][MT > 0 ? MT : 1];
  if constexpr (MT > 0) {
#pragma unroll
    for (int p = 0; p < MT; ++p) th[0][p] = ld4(at_elem(pl + p * S, plo));
  }
  // The solved rows of tile i for the workgroup's units, staged in LDS
  // (zl[unit][k][column], zeros past each unit's columns, negated: the
  // products are subtracted), all loads in flight together.  Thread
  // (row r0 = tid / 16, column cc = tid % 16) takes rows r0 + 16 n of every
  // unit.
  {
    const int cc = threadIdx.x & 15, r0 = threadIdx.x >> 4;
    const double* srow = src + (m * dp + (int64_t)i * NB) * ldz;
    unsigned so[U];
    bool sok[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int u = g * U + j;
      const int uc = u < nunits ? u : nunits - 1;
      const int t = uc / ncu, h = uc - t * ncu;
      const int ncol = (c - 16 * h) < 16 ? (c - 16 * h) : 16;
      sok[j] = u < nunits && cc < ncol;
      so[j] = (unsigned)(r0 * ldzi + t * c + 16 * h + (cc < ncol ? cc : ncol - 1));
    }
    double v[U][8];
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int n = 0; n < 8; ++n) v[j][n] = *at_elem(srow + (int64_t)16 * n * ldz, so[j]);
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int n = 0; n < 8; ++n)
        zl[((j * NB + r0 + 16 * n) << 4) + cc] = sok[j] ? -v[j][n] : 0.0;
  }
  __syncthreads();
  const double* zb = zl + ((kb + lq) << 4) + lr;  // B(k, lane column) of unit 0
  if constexpr (MT > 0) {
    // the coefficient values of each k step are loaded two steps before
    // its products (three register sets; the 16 steps are unrolled, and
    // scheduling barriers keep the compiler from moving products ahead of
    // loads issued after them, which would make them wait for those loads)
    auto load = [&](int k0, v4d (&t)[MT]) {
      const double* pk = pl + (int64_t)k0 * NB;
#pragma unroll
      for (int p = 0; p < MT; ++p) t[p] = ld4(at_elem(pk + p * S, plo));
    };
    auto step = [&](int k0, const v4d (&t)[MT]) {
#pragma unroll
      for (int j = 0; j < U; ++j) {
        v4d a = t[MT - 1];
#pragma unroll
        for (int p = MT - 2; p >= 0; --p) a = a * tv[j] + t[p];
        const double b = zb[(j * NB + k0) << 4];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
          acc[j][bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b, acc[j][bi], 0, 0, 0);
      }
    };
    load(4, th[1]);
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      if (st + 2 < 16) load(4 * (st + 2), th[(st + 2) % 3]);
      __builtin_amdgcn_sched_barrier(0);
      step(4 * st, th[st % 3]);
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll 1
    for (int k0 = 0; k0 < 64; k0 += 4) {
      const double* pk = pl + (int64_t)k0 * NB;
      v4d a[U];
      v4d th = ld4(at_elem(pk + (int64_t)(M - 1) * S, plo));
#pragma unroll
      for (int j = 0; j < U; ++j) a[j] = th;
      for (int p = M - 2; p >= 0; --p) {
        th = ld4(at_elem(pk + (int64_t)p * S, plo));
#pragma unroll
        for (int j = 0; j < U; ++j) a[j] = a[j] * tv[j] + th;
      }
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const double b = zb[(j * NB + k0) << 4];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
          acc[j][bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j][bi], b, acc[j][bi],
                                                            0, 0, 0);
      }
    }
  }
  __syncthreads();  // every wave is done with the staged rows
  // the second k half's partial sums to the first (LDS, fixed order)
  auto zidx = [&](int j, int v, int bi) {
    return ((j * NB + rh * 64 + 16 * v + 4 * lq + bi) << 4) + lr;
  };
  if (kh == 1) {
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) zl[zidx(j, v, bi)] = acc[j][bi][v];
  }
  __syncthreads();
  if (kh == 0) {
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[j][bi][v] += zl[zidx(j, v, bi)];
    if (ro != 0) {
#pragma unroll
      for (int j = 0; j < U; ++j)
        if (ok[j])
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              *at_elem(drow + (int64_t)(16 * v + bi) * ldz, dro[j]) = acc[j][bi][v];
    } else {
      // the updated block, whole, for the diagonal solve below (each lane
      // overwrites only the entries it has just read)
#pragma unroll
      for (int j = 0; j < U; ++j)
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
          for (int v = 0; v < 4; ++v) zl[zidx(j, v, bi)] = acc[j][bi][v];
    }
  }
  if (ro != 0) return;
  __syncthreads();
  // fused diagonal solve of tile row I: wave (rh, kh) forms the rows of
  // half rh for the units 2kh, 2kh + 1
  constexpr int UH = U / 2;
  v4d ac2[UH][4];
#pragma unroll
  for (int j = 0; j < UH; ++j)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) ac2[j][bi] = v4d{0.0, 0.0, 0.0, 0.0};
  const double* lbase = dinv + ((m * q) * nt + I) * (int64_t)NB2;
  unsigned lvo[UH];  // offset of the unit's inverse from lbase
#pragma unroll
  for (int j = 0; j < UH; ++j) lvo[j] = (unsigned)(tt[kh * UH + j] * nt * NB2);
  // The inverse is read in chunks of 32 k, all of a chunk's loads issued
  // before its products (the accumulators of the update are free by now).
  if (FWD) {
    // row r of the inverse is zero beyond column r: half rh needs k < 64(rh+1)
    const int kend = 64 * (rh + 1);
    const unsigned ao = (unsigned)(rh * 64 + 4 * lr + lq * NB);
#pragma unroll 1
    for (int kc = 0; kc < kend; kc += 32) {
      v4d a[8][UH];
#pragma unroll
      for (int st = 0; st < 8; ++st)
#pragma unroll
        for (int j = 0; j < UH; ++j)
          a[st][j] = ld4(at_elem(lbase + (kc + 4 * st) * NB, lvo[j] + ao));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int st = 0; st < 8; ++st)
#pragma unroll
        for (int j = 0; j < UH; ++j) {
          const double b = zl[(((kh * UH + j) * NB + kc + 4 * st + lq) << 4) + lr];
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
            ac2[j][bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st][j][bi], b, ac2[j][bi],
                                                              0, 0, 0);
        }
    }
  } else {
    // the transpose: A(row, k) = Linv(k, row) at row * 128 + k, nonzero for
    // k >= row, so half rh needs k >= 64 rh.  Four consecutive k of a row per
    // 32-byte load: in step s of a 16-long block lane group lq supplies
    // k = k0 + 4 lq + s, and the B operand follows that order.
    const unsigned ao = (unsigned)((rh * 64 + 4 * lr) * NB + 4 * lq);
#pragma unroll 1
    for (int kc = 64 * rh; kc < NB; kc += 32) {
      v4d a[2][UH][4];
#pragma unroll
      for (int hb = 0; hb < 2; ++hb)
#pragma unroll
        for (int j = 0; j < UH; ++j)
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
            a[hb][j][bi] = ld4(at_elem(lbase + bi * NB + kc + 16 * hb, lvo[j] + ao));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int hb = 0; hb < 2; ++hb)
#pragma unroll
        for (int j = 0; j < UH; ++j)
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const double b =
                zl[(((kh * UH + j) * NB + kc + 16 * hb + 4 * lq + s4) << 4) + lr];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
              ac2[j][bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[hb][j][bi][s4], b,
                                                                ac2[j][bi], 0, 0, 0);
          }
    }
  }
  double* orow = out + (m * dp + (int64_t)I * NB + rh * 64) * ldz;
#pragma unroll
  for (int j = 0; j < UH; ++j)
    if (ok[kh * UH + j])
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          *at_elem(orow + (int64_t)(16 * v + bi) * ldz, dro[kh * UH + j]) = ac2[j][bi][v];
}

// Off-diagonal update for exact factors, one factor per lambda t:
// forward rows of tile I > i lose L_t(I,i) U_i, backward rows of tile I < i
// lose L_t(i,I)^T W_i, on FP64 MFMA.  A workgroup of two waves takes one
// (tile, lambda): each wave a 64-row half of the result and the lambda's c
// columns in groups of 16 (v_mfma_f64_16x16x4 blocks; B lanes past c read
// zeros).  Forward: one 32-byte load of four consecutive rows of L per lane
// and k step feeds the four row blocks.  Backward: the transposed tile is
// read along its columns, four consecutive k of one row per 32-byte load,
// so a lane group supplies k = 4*lq + s in step s of each 16-long chunk and
// the B lanes follow the same order.  The kernel streams every factor tile
// once per step (HBM-bound).
template <bool FWD>
__global__ void __launch_bounds__(128) k_update_factors(int64_t d, int i,
                                                        const double* L,
                                                        int64_t S, int nper,
                                                        int c, int64_t ldz,
                                                        const double* Xs,
                                                        double* Z) {
  const int I = FWD ? i + 1 + (int)blockIdx.x : (int)blockIdx.x;
  const int t = blockIdx.y;
  const int64_t m = blockIdx.z;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lq = l >> 4, lr = l & 15;
  const int64_t dp = ntiles_of(d) * NB;
  const double* tile = L + (m * nper + t) * S + (FWD ? tile_off(I, i) : tile_off(i, I));
  // the solved block rows of tile i (in Xs) and the rows of tile I (in Z)
  const double* zsrc = Xs + (m * dp + (int64_t)i * NB) * ldz + (int64_t)t * c;
  double* zdst = Z + (m * dp + (int64_t)I * NB + w * 64) * ldz + (int64_t)t * c;
  for (int cg = 0; cg < c; cg += 16) {
    const bool cok = cg + lr < c;
    v4d acc[4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) acc[bi] = v4d{0.0, 0.0, 0.0, 0.0};
    if (FWD) {
      // A(n, k) = L(I,i)(w*64 + n, k) at k*128 + w*64 + n
      const double* pa = tile + (int64_t)lq * NB + w * 64 + 4 * lr;
      const double* pb = zsrc + (int64_t)lq * ldz + cg + lr;
      // four groups of eight k steps, all of a group's loads issued before
      // its products: sixteen loads per lane in flight at occupancy two
#pragma unroll 1
      for (int h = 0; h < 4; ++h) {
        v4d av[8];
        double bv[8];
#pragma unroll
        for (int st = 0; st < 8; ++st) {
          const int k0 = 32 * h + 4 * st;
          av[st] = ld4(pa + (int64_t)k0 * NB);
          bv[st] = cok ? pb[(int64_t)k0 * ldz] : 0.0;
        }
#pragma unroll
        for (int st = 0; st < 8; ++st)
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
            acc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st][bi], bv[st], acc[bi], 0, 0, 0);
      }
    } else {
      // A(n, k) = L(i,I)(k, w*64 + n) at (w*64 + n)*128 + k
#pragma unroll 2
      for (int k0 = 0; k0 < NB; k0 += 16) {
        v4d av[4];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
          av[bi] = ld4(tile + (int64_t)(w * 64 + 4 * lr + bi) * NB + k0 + 4 * lq);
        double bv[4];
#pragma unroll
        for (int sk = 0; sk < 4; ++sk)
          bv[sk] = cok ? zsrc[(int64_t)(k0 + 4 * lq + sk) * ldz + cg + lr] : 0.0;
#pragma unroll
        for (int sk = 0; sk < 4; ++sk)
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
            acc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi][sk], bv[sk], acc[bi], 0, 0, 0);
      }
    }
    // element v of block bi: row 16v + 4lq + bi of the half, column lr;
    // the sixteen slab values are all loaded before any is stored
    if (cok) {
      double cur[4][4];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
          cur[v][bi] = zdst[(int64_t)(16 * v + 4 * lq + bi) * ldz + cg + lr];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
          zdst[(int64_t)(16 * v + 4 * lq + bi) * ldz + cg + lr] =
              cur[v][bi] - acc[bi][v];
    }
  }
}

static hipError_t slab_init(int64_t d, int nmat, int q, int c, int64_t ldz,
                            const double* B, double* Z, int* flags,
                            hipStream_t s) {
  const int64_t dp = ntiles_of(d) * NB;
  unsigned bx = (unsigned)((dp * ldz + 255) / 256);
  if (bx > 4096) bx = 4096;
  PICHOL_LAUNCH(k_slab_init, dim3(bx, (unsigned)nmat), dim3(256), 0, s,
                     dp, q, c, ldz, B, Z, flags);
  return hipGetLastError();
}

hipError_t launch_slab_init(int64_t d, int nmat, int q, int c, int64_t ldz,
                            const double* B, double* Z, int* flags,
                            hipStream_t s) {
  return slab_init(d, nmat, q, c, ldz, B, Z, flags, s);
}

// Forward steps take the right-hand sides from Z and leave the solved
// blocks in X; back steps take them from X and leave the solution in Z.
// Each diagonal apply reads one slab and writes the other, so its four
// workgroups per (fold, lambda) never overwrite rows another one reads.
// The inverted diagonal blocks of tile rows i0 .. i1-1 of every
// interpolated factor (k_diag_inv).
hipError_t launch_diag_inv(int64_t d, int nmat, int M, const double* theta,
                           int q, const double* tau_dev, double* dinv,
                           int* flags, int i0, int i1, hipStream_t s) {
  const int nt = (int)ntiles_of(d);
  if (i0 < 0 || i1 > nt || i0 > i1) return hipErrorInvalidValue;
  if (i0 == i1) return hipSuccess;
  FactorSrc src{theta, packed_elems_of(d), M, 0, q, tau_dev};
  PICHOL_LAUNCH(k_diag_inv,
                dim3((unsigned)(i1 - i0), (unsigned)q, (unsigned)nmat),
                dim3(256), 0, s, d, src, dinv, flags, i0);
  return hipGetLastError();
}


// Launches of the per-lambda step with fewer workgroups than this at four
// units each take two units per workgroup, and so do all launches with
// `narrow` (steps that share the GPU with nothing else: the four-unit form
// disturbs a concurrent factorization less, the two-unit one finishes a
// lone step sooner).
constexpr int STEP_SMALL_LAUNCH = 512;

template <bool FWD>
static hipError_t step_interp(int M, int nrows, hipStream_t s, int64_t d, int i,
                              int nmat, const double* theta, int64_t S, int q,
                              int c, const double* tau, int64_t ldz,
                              const double* dinv, const double* src,
                              double* dst, double* out, bool narrow) {
  const int nunits = q * ((c + 15) / 16);
  const int g4 = (nunits + 3) / 4;
  const bool small = narrow || (int64_t)nmat * nrows * g4 < STEP_SMALL_LAUNCH;
  const int ngrp = small ? (nunits + 1) / 2 : g4;
  const dim3 grid((unsigned)(nmat * nrows * ngrp));
#define PICHOL_STEP(MT, U)                                                      \
  PICHOL_LAUNCH((k_step_interp<FWD, MT, U>), grid, dim3(256), 0, s, d, i, nmat, \
                theta, S, M, q, c, tau, ldz, nrows, ngrp, dinv, src, dst, out)
  if (small) {
    switch (M) {
      case 1: PICHOL_STEP(1, 2); break;
      case 2: PICHOL_STEP(2, 2); break;
      case 3: PICHOL_STEP(3, 2); break;
      default: PICHOL_STEP(0, 2); break;
    }
  } else {
    switch (M) {
      case 1: PICHOL_STEP(1, 4); break;
      case 2: PICHOL_STEP(2, 4); break;
      case 3: PICHOL_STEP(3, 4); break;
      default: PICHOL_STEP(0, 4); break;
    }
  }
#undef PICHOL_STEP
  return hipGetLastError();
}

// Forward steps i0 .. i1-1 of the per-lambda form (i0 = 0 starts with the
// first diagonal block): afterwards the solved blocks 0 .. i1 are in X and
// the rows below block i1 have received blocks 0 .. i1-1.  Step i reads the
// coefficient tiles of column i and the inverted diagonal block i+1 only.
hipError_t launch_solve_fwd(int64_t d, int nmat, int c, int M,
                            const double* theta, int q, const double* tau_dev,
                            int64_t ldz, double* Z, double* X,
                            const double* dinv, int i0, int i1, hipStream_t s,
                            bool narrow) {
  const int nt = (int)ntiles_of(d);
  const int64_t S = packed_elems_of(d);
  if (i0 < 0 || i1 > nt - 1 || i0 > i1) return hipErrorInvalidValue;
  if (i0 == 0)
    PICHOL_LAUNCH(k_diag_apply<true>, dim3((unsigned)(4 * q), (unsigned)nmat),
                  dim3(256), 0, s, d, 0, q, c, dinv, ldz, Z, X);
  for (int i = i0; i < i1; ++i) {
    const hipError_t e = step_interp<true>(M, nt - i - 1, s, d, i, nmat, theta, S,
                                           q, c, tau_dev, ldz, dinv, X, Z, X,
                                           narrow);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

int solve_form_for(int M, int q, int c, int64_t ldz, int requested) {
  if (requested == 0) requested = option_solve_form();
  if (requested == 1 || requested == 2) return requested;
  // automatic: per step and tile, the stacked product runs over M * ldz
  // columns (K = 128 per plane), the per-lambda one over 16 * q * ncu (each
  // lambda's columns padded to 16); the per-lambda kernel also evaluates
  // its operands and reaches about two thirds of the stacked one's rate
  const int64_t ncu = (c + 15) / 16;
  return (int64_t)M * ldz >= 24 * (int64_t)q * ncu ? 2 : 1;
}

hipError_t launch_solve_interp(int64_t d, int nmat, int c, int M,
                               const double* theta, const double* theta_t,
                               int q, const double* tau_dev, int64_t ldz,
                               double* Z, double* X, int* flags, double* dinv,
                               int prepare, hipStream_t s, int fwd_from,
                               int form) {
  const int nt = (int)ntiles_of(d);
  const int64_t S = packed_elems_of(d);
  const unsigned ncb = (unsigned)(ldz / NB);
  if (prepare) {
    const hipError_t e =
        launch_diag_inv(d, nmat, M, theta, q, tau_dev, dinv, flags, 0, nt, s);
    if (e != hipSuccess) return e;
  }
  const dim3 agrid((unsigned)(4 * q), (unsigned)nmat);
  if (solve_form_for(M, q, c, ldz, form) == 1) {
    // stacked form: a diagonal launch and an update launch per step
    for (int i = 0; i < nt; ++i) {
      PICHOL_LAUNCH(k_diag_apply<true>, agrid, dim3(256), 0, s, d, i, q, c, dinv,
                    ldz, Z, X);
      if (i + 1 < nt) {
        const int nrows = nt - i - 1;
        PICHOL_LAUNCH(k_update_interp<true>, dim3(ncb * 2 * nrows * nmat),
                      dim3(256), 0, s, d, i, theta, theta_t, S, M, q, c, tau_dev,
                      ldz, (int)ncb, nrows, X, Z);
      }
    }
    for (int i = nt - 1; i >= 0; --i) {
      PICHOL_LAUNCH(k_diag_apply<false>, agrid, dim3(256), 0, s, d, i, q, c,
                    dinv, ldz, X, Z);
      if (i > 0)
        PICHOL_LAUNCH(k_update_interp<false>, dim3(ncb * 2 * i * nmat), dim3(256),
                      0, s, d, i, theta, theta_t, S, M, q, c, tau_dev, ldz,
                      (int)ncb, i, Z, X);
    }
    return hipGetLastError();
  }
  // per-lambda form: the first diagonal block of each sweep on its own,
  // every other one inside the step that completes it
  const hipError_t ef = launch_solve_fwd(d, nmat, c, M, theta, q, tau_dev, ldz,
                                         Z, X, dinv, fwd_from, nt - 1, s, true);
  if (ef != hipSuccess) return ef;
  PICHOL_LAUNCH(k_diag_apply<false>, agrid, dim3(256), 0, s, d, nt - 1, q, c,
                dinv, ldz, X, Z);
  for (int i = nt - 1; i > 0; --i) {
    const hipError_t e = step_interp<false>(M, i, s, d, i, nmat, theta_t, S, q, c,
                                            tau_dev, ldz, dinv, Z, X, Z, true);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_solve_factors(int64_t d, int nmat, int nper, int c,
                                const double* L, int64_t ldz, double* Z,
                                int* flags, const double* linv, double* X,
                                hipStream_t s) {
  const int nt = (int)ntiles_of(d);
  const int64_t S = packed_elems_of(d);
  if (linv && X) {
    // as for interpolated factors: forward steps take the right-hand sides
    // from Z and leave the solved blocks in X, back steps the reverse
    const dim3 agrid((unsigned)(4 * nper), (unsigned)nmat);
    for (int i = 0; i < nt; ++i) {
      PICHOL_LAUNCH(k_diag_apply<true>, agrid, dim3(256), 0, s, d, i, nper, c,
                    linv, ldz, Z, X);
      if (i + 1 < nt)
        PICHOL_LAUNCH(k_update_factors<true>,
                      dim3((unsigned)(nt - i - 1), (unsigned)nper, (unsigned)nmat),
                      dim3(128), 0, s, d, i, L, S, nper, c, ldz, X, Z);
    }
    for (int i = nt - 1; i >= 0; --i) {
      PICHOL_LAUNCH(k_diag_apply<false>, agrid, dim3(256), 0, s, d, i, nper, c,
                    linv, ldz, X, Z);
      if (i > 0)
        PICHOL_LAUNCH(k_update_factors<false>,
                      dim3((unsigned)i, (unsigned)nper, (unsigned)nmat),
                      dim3(128), 0, s, d, i, L, S, nper, c, ldz, Z, X);
    }
    return hipGetLastError();
  }
  FactorSrc src{L, S, 1, 1, nper, nullptr};
  for (int i = 0; i < nt; ++i) {
    PICHOL_LAUNCH(k_diag_solve<true>, dim3((unsigned)nper, (unsigned)nmat),
                       dim3(256), 0, s, d, i, src, c, ldz, Z, flags);
    if (i + 1 < nt)
      PICHOL_LAUNCH(k_update_factors<true>,
                    dim3((unsigned)(nt - i - 1), (unsigned)nper, (unsigned)nmat),
                    dim3(128), 0, s, d, i, L, S, nper, c, ldz, Z, Z);
  }
  for (int i = nt - 1; i >= 0; --i) {
    PICHOL_LAUNCH(k_diag_solve<false>, dim3((unsigned)nper, (unsigned)nmat),
                       dim3(256), 0, s, d, i, src, c, ldz, Z, flags);
    if (i > 0)
      PICHOL_LAUNCH(k_update_factors<false>,
                    dim3((unsigned)i, (unsigned)nper, (unsigned)nmat),
                    dim3(128), 0, s, d, i, L, S, nper, c, ldz, Z, Z);
  }
  return hipGetLastError();
}

}  // namespace pichol
