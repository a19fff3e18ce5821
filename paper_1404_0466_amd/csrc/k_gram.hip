// Fold Gram matrices (Sec. 3.1: H = X^T X, g = X^T y) for k-fold
// cross-validation.  Each fold's validation block b contributes
// G_b = X_b^T X_b and C_b = X_b^T Y_b; the training Gram of fold f is the sum
// of the other blocks, so no cancellation occurs.
#include <algorithm>
#include <atomic>

#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

__device__ inline v4d ld4_masked(const double* rowp, int64_t col, int64_t d,
                                 bool row_ok) {
  v4d v = {0.0, 0.0, 0.0, 0.0};
  if (row_ok) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (col + e < d) v[e] = rowp[col + e];
  }
  return v;
}

// Tile t of the lower triangle of nt x nt tiles in the Gram kernel's order:
// the triangle is cut into 8 x 8 blocks of tiles (the diagonal blocks keep
// their lower half), taken block row by block row, and each block's tiles
// row by row.  The 64 tiles of one block read 8 column strips of X per
// operand, where 64 tiles taken row by row along the triangle read about 2
// strips each.
__device__ inline void gram_tile_of(int t, int nt, int& I, int& J) {
  constexpr int SB = 8;
  for (int P = 0; P * SB < nt; ++P) {
    const int r0 = P * SB, rs = nt - r0 < SB ? nt - r0 : SB;
    for (int Q = 0; Q <= P; ++Q) {
      const int c0 = Q * SB;
      const int n = Q == P ? rs * (rs + 1) / 2 : rs * SB;
      if (t < n) {
        if (Q == P) {
          const int i = tri_row(t);
          I = r0 + i;
          J = c0 + (t - (int)tri(i));
        } else {
          const int i = t / SB;
          I = r0 + i;
          J = c0 + (t - i * SB);
        }
        return;
      }
      t -= n;
    }
  }
  I = J = 0;  // not reached for t < tri(nt)
}

// The wave's 64 x 64 part of a Gram tile summed over rows ra .. rb-1 of X:
// D'(n,m) += sum_r X[r][ncol+n] X[r][mcol+m] on FP64 MFMA.
__device__ inline void gram_rows(Acc64& acc, const double* X, int64_t ldx,
                                 int64_t d, int64_t ncol, int64_t mcol,
                                 int64_t ra, int64_t rb, int vec_ok) {
  const LaneXY lx;
  const int64_t K = rb - ra;
  const bool fast = vec_ok && ncol + 64 <= d && mcol + 64 <= d;
  int64_t kdone = 0;
  if (fast && K >= 4) {
    const int64_t K4 = K & ~(int64_t)3;
    // mma_panel takes an int K; split very long blocks into chunks
    for (int64_t k0 = 0; k0 < K4; k0 += (1 << 28)) {
      int kk = (int)((K4 - k0) < (1 << 28) ? (K4 - k0) : (1 << 28));
      mma_panel(acc, X + (ra + k0) * ldx + ncol, ldx,
                X + (ra + k0) * ldx + mcol, ldx, kk);
    }
    kdone = K4;
  }
  // remaining rows (all rows on the masked path), four at a time
  for (int64_t k0 = kdone; k0 < K; k0 += 4) {
    const int64_t r = ra + k0 + lx.lq;
    const bool ok = r < rb;
    const double* rowp = X + (ok ? r : ra) * ldx;
    v4d av = ld4_masked(rowp, ncol + lx.col0(), d, ok);
    v4d bv = ld4_masked(rowp, mcol + lx.col0(), d, ok);
    acc.mma(av, bv);
  }
}

// G_b tile (I,J), J <= I, over the rows of block b; FP64 MFMA.  The wave
// computes D'(n,m) = sum_r X[r][J*128+n] X[r][I*128+m] for its 64 x 64 part,
// i.e. G(I*128+m, J*128+n), which is element n*128+m of the column-major tile
// (I,J); the mirror tile (J,I) receives the transpose.
// Tiles are numbered block by block, then in gram_tile_of's order.  The
// first nmain workgroups take tiles 0 .. nmain-1 whole, spread over the XCDs
// in contiguous ranges so that the workgroups running together on one XCD
// stream the same few strips of X through its L2.  When the tile count is
// not a multiple of the workgroups the GPU holds at once, the last ntail
// tiles would run as a thin final round; they are cut instead into nsplit
// chunks of their block's rows, one workgroup per (chunk, tile) after the
// whole tiles, each writing its partial tile (column-major, the chunk-major
// order of the workgroups) to part for k_gram_tail to add up.
__global__ void __launch_bounds__(256) k_gram_tiles(const double* X,
                                                    int64_t ldx, int64_t d,
                                                    int64_t nt, FoldSplit fs,
                                                    double* G, int vec_ok,
                                                    int nmain, int ntail,
                                                    int nsplit, double* part) {
  const int ntri = (int)tri(nt);
  const int u = (int)blockIdx.x;
  const bool whole = u < nmain;
  int tl, p = 0;
  if (whole) {
    tl = xcd_remap(u, nmain);
  } else {
    p = (u - nmain) / ntail;
    tl = nmain + (u - nmain - p * ntail);
  }
  const int b = tl / ntri;
  int I, J;
  gram_tile_of(tl - b * ntri, (int)nt, I, J);
  const int w = threadIdx.x >> 6, wi = w >> 1, wj = w & 1;
  int64_t ra = fs.start[b], rb = fs.start[b + 1];
  if (!whole) {
    // chunk p of the block's rows, a multiple of four rows long
    const int64_t kc = ((rb - ra + nsplit - 1) / nsplit + 3) & ~(int64_t)3;
    const int64_t a0 = ra + p * kc;
    const int64_t a1 = a0 + kc;
    ra = a0 < rb ? a0 : rb;
    rb = a1 < rb ? a1 : rb;
  }
  const int64_t ncol = (int64_t)J * NB + wi * 64;  // A' columns of X
  const int64_t mcol = (int64_t)I * NB + wj * 64;  // B' columns of X
  const LaneXY lx;

  Acc64 acc;
  acc.zero();
  gram_rows(acc, X, ldx, d, ncol, mcol, ra, rb, vec_ok);

  double* gb = G + (int64_t)b * nt * nt * NB2;
  double* gt = whole ? gb + ((int64_t)I * nt + J) * NB2
                     : part + (int64_t)(u - nmain) * NB2;
  double* gm = gb + ((int64_t)J * nt + I) * NB2;
  const int m0 = wj * 64 + lx.col0();
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const int n = wi * 64 + lx.row(v, bi);
      const v4d val = acc.row(v, bi);
      st4(gt + n * NB + m0, val);
      if (whole && I != J) {
#pragma unroll
        for (int e = 0; e < 4; ++e) gm[(m0 + e) * NB + n] = val[e];
      }
    }
}

// The split tiles of k_gram_tiles: tile nmain + j is the sum of its nsplit
// (at most 8) partial tiles, added in chunk order, written with its mirror.
// Workgroup (j, y) takes elements y*1024 .. y*1024+1023 of the tile, four
// consecutive ones per thread, with the loads of every chunk in flight
// together.
constexpr int GRAM_SPLIT_MAX = 8;
__global__ void __launch_bounds__(256) k_gram_tail(int64_t nt, int nmain,
                                                   int ntail, int nsplit,
                                                   const double* part,
                                                   double* G) {
  const int ntri = (int)tri(nt);
  const int j = (int)blockIdx.x;
  const int tl = nmain + j;
  const int b = tl / ntri;
  int I, J;
  gram_tile_of(tl - b * ntri, (int)nt, I, J);
  double* gb = G + (int64_t)b * nt * nt * NB2;
  double* gt = gb + ((int64_t)I * nt + J) * NB2;
  double* gm = gb + ((int64_t)J * nt + I) * NB2;
  const int e = (int)blockIdx.y * 1024 + 4 * (int)threadIdx.x;
  v4d v[GRAM_SPLIT_MAX];
#pragma unroll
  for (int p = 0; p < GRAM_SPLIT_MAX; ++p)
    if (p < nsplit) v[p] = ld4(part + ((int64_t)p * ntail + j) * NB2 + e);
  v4d acc = v[0];
#pragma unroll
  for (int p = 1; p < GRAM_SPLIT_MAX; ++p)
    if (p < nsplit) acc += v[p];
  st4(gt + e, acc);
  // element e = n*128 + m of the tile is element m*128 + n of its mirror
  if (I != J) {
    const int n = e >> 7, m = e & (NB - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) gm[(m + q) * NB + n] = acc[q];
  }
}

// C_b = X_b^T Y_b (dp x c, row-major, padding rows 0) on FP64 MFMA.  A
// workgroup takes 64 rows i of C_b (64 columns of X) and 16 columns of Y at
// a time; its four wavefronts sum over consecutive quarters of the block's
// rows, then the quarters are added in a fixed order through LDS.  A lane
// loads four consecutive columns of one row of X (32 bytes) per k step,
// feeding the four 16-row blocks; B lanes past c read zeros.  Eight k steps
// are issued together so that the stream of X keeps many loads in flight.
// The workgroups of the first 64 rows also return yy[b], the sum of squares
// of Y over the block (each element of Y_b is loaded once by one lane; the
// lanes' sums are added in a fixed tree).
__global__ void __launch_bounds__(256) k_gram_rhs(const double* X, int64_t ldx,
                                                  const double* Y, int64_t ldy,
                                                  int64_t d, int64_t c,
                                                  int64_t dp, FoldSplit fs,
                                                  int vec_ok, double* C,
                                                  double* yy) {
  __shared__ v4d part[3][4][64];
  __shared__ double red[256];
  double ysq = 0.0;
  const int b = blockIdx.y;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lq = l >> 4, lr = l & 15;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int64_t r0 = fs.start[b], r1 = fs.start[b + 1];
  const int64_t nq = ((r1 - r0 + 3) / 4 + 3) / 4 * 4;  // rows per quarter
  const int64_t q0 = r0 + w * nq;
  const int64_t q1 = (q0 + nq < r1) ? q0 + nq : r1;
  const int64_t col = i0 + 4 * lr;
  const bool fast = vec_ok && i0 + 64 <= d;
  for (int64_t cg = 0; cg < c; cg += 16) {
    const bool cok = cg + lr < c;
    v4d acc[4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) acc[bi] = v4d{0.0, 0.0, 0.0, 0.0};
    int64_t r = q0;
    if (fast) {
      for (; r + 32 <= q1; r += 32) {
        v4d av[8];
        double bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t rr = r + 4 * u + lq;
          av[u] = ld4(X + rr * ldx + col);
          bv[u] = cok ? Y[rr * ldy + cg + lr] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) ysq += bv[u] * bv[u];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int bi = 0; bi < 4; ++bi)
            acc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][bi], bv[u], acc[bi], 0, 0, 0);
      }
    }
    // remaining rows of the quarter (all rows when not vectorizable)
    for (; r < q1; r += 4) {
      const int64_t rr = r + lq;
      const bool ok = rr < q1;
      v4d av = {0.0, 0.0, 0.0, 0.0};
      if (ok) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (col + e < d) av[e] = X[rr * ldx + col + e];
      }
      const double bv = (ok && cok) ? Y[rr * ldy + cg + lr] : 0.0;
      ysq += bv * bv;
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
        acc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], bv, acc[bi], 0, 0, 0);
    }
    if (cg) __syncthreads();  // the previous group's partial sums were read
    if (w > 0) {
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) part[w - 1][bi][l] = acc[bi];
    }
    __syncthreads();
    if (w == 0 && cok) {
      // element v of block bi: row 16v + 4lq + bi of the 64, column lr
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) {
        const v4d s1 = part[0][bi][l], s2 = part[1][bi][l], s3 = part[2][bi][l];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t i = i0 + 16 * v + 4 * lq + bi;
          C[((int64_t)b * dp + i) * c + cg + lr] =
              ((acc[bi][v] + s1[v]) + s2[v]) + s3[v];
        }
      }
    }
  }
  if (blockIdx.x == 0) {
    const int tid = threadIdx.x;
    red[tid] = ysq;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) yy[b] = red[0];
  }
}

// H_f = scale_f * sum_{b != f} G_b on the lower tiles, the blocks added in
// increasing order; padding gets the identity.  With at most KM folds a
// workgroup takes a quarter of one tile for every fold at once: each
// element of the k blocks is read once into registers and every fold's sum
// is formed from them.  With more folds, blockIdx.y is the fold and each
// fold's workgroups read the blocks again.
template <int KM>
__global__ void __launch_bounds__(256) k_gram_combine_h(int64_t d, int64_t nt,
                                                        FoldSplit fs,
                                                        const double* G,
                                                        double* H, int64_t S) {
  const int I = tri_row(blockIdx.x), J = blockIdx.x - (int)tri(I);
  const int64_t gstride = nt * nt * NB2;
  const double* g0 = G + ((int64_t)I * nt + J) * NB2;
  const int64_t hoff = tile_off(I, J);
  const int k = fs.k;
  const int e0 = KM > 0 ? (int)blockIdx.y * (NB2 / 4) : 0;
  const int e1 = KM > 0 ? e0 + NB2 / 4 : NB2;
  for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) {
    const int64_t i = (int64_t)I * NB + (e & (NB - 1));
    const int64_t j = (int64_t)J * NB + (e >> 7);
    const bool pad = i >= d || j >= d;
    if (KM > 0) {
      double v[KM > 0 ? KM : 1];
#pragma unroll
      for (int b = 0; b < KM; ++b)
        v[b] = (b < k && !pad) ? g0[b * gstride + e] : 0.0;
#pragma unroll
      for (int f = 0; f < KM; ++f) {
        if (f >= k) break;
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < KM; ++b)
          if (b < k && b != f) acc += v[b];
        H[f * S + hoff + e] = pad ? (i == j ? 1.0 : 0.0) : acc * fs.scale[f];
      }
    } else {
      const int f = blockIdx.y;
      double acc = 0.0;
      if (!pad)
        for (int b = 0; b < k; ++b)
          if (b != f) acc += g0[b * gstride + e];
      H[f * S + hoff + e] = pad ? (i == j ? 1.0 : 0.0) : acc * fs.scale[f];
    }
  }
}

// B_f = scale_f * sum_{b != f} C_b.
__global__ void __launch_bounds__(256) k_gram_combine_b(int64_t n_el,
                                                        FoldSplit fs,
                                                        const double* C,
                                                        double* B) {
  const int f = blockIdx.y;
  const double sc = fs.scale[f];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_el;
       e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < fs.k; ++b)
      if (b != f) acc += C[b * n_el + e];
    B[f * n_el + e] = acc * sc;
  }
}

// Workgroups of k_gram_tiles the current device runs at once (0 if
// unknown), looked up once per device.
static int gram_slots() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    int cu = 0, per = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount,
                              dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_gram_tiles, 256,
                                                     0) != hipSuccess)
      cu = per = 0;
    v = cu * per > 0 ? cu * per : -1;
    cache[dev].store(v, std::memory_order_relaxed);
  }
  return v > 0 ? v : 0;
}

void prepare_gram() { (void)gram_slots(); }

// Row chunks for the tiles of the last, partly filled round of
// k_gram_tiles: the count s (1 = no split) that minimises that round's
// length ceil(tail*s / slots) / s in whole-tile times.  The tail*s partial
// tiles must fit in H (one tile of H per Gram tile) and each chunk keeps at
// least 256 rows.
static int gram_split(int ntiles, int slots, int64_t kmin) {
  if (slots <= 0) return 1;
  const int tail = ntiles % slots;
  if (tail == 0) return 1;
  int best = 1;
  double best_len = 1.0;
  for (int sp = 2; sp <= GRAM_SPLIT_MAX; ++sp) {
    if ((int64_t)tail * sp > ntiles || kmin / sp < 256) break;
    const double len = (double)((tail * sp + slots - 1) / slots) / sp;
    if (len < best_len) {
      best_len = len;
      best = sp;
    }
  }
  return best;
}

hipError_t launch_gram(const double* X, int64_t ldx, const double* Y,
                       int64_t ldy, int64_t d, int64_t c,
                       const FoldSplit& fs, double* G, double* C, double* yy,
                       double* H, double* B, hipStream_t s) {
  const int64_t nt = ntiles_of(d), dp = nt * NB, S = packed_elems_of(d);
  const int vec_ok = ((ldx & 3) == 0) && ((((uintptr_t)X) & 31) == 0);
  const int ntiles = (int)tri(nt) * fs.k;
  int64_t kmin = fs.start[1] - fs.start[0];
  for (int b = 1; b < fs.k; ++b)
    kmin = std::min<int64_t>(kmin, fs.start[b + 1] - fs.start[b]);
  const int nsplit = gram_split(ntiles, gram_slots(), kmin);
  const int ntail = nsplit > 1 ? ntiles % gram_slots() : 0;
  const int nmain = ntiles - ntail;
  // the partial tiles live in H until k_gram_combine_h writes it
  PICHOL_LAUNCH(k_gram_tiles, dim3((unsigned)(nmain + ntail * nsplit)),
                dim3(256), 0, s, X, ldx, d, nt, fs, G, vec_ok, nmain, ntail,
                nsplit, H);
  if (ntail > 0)
    PICHOL_LAUNCH(k_gram_tail, dim3((unsigned)ntail, NB2 / 1024), dim3(256), 0,
                  s, nt, nmain, ntail, nsplit, H, G);
  PICHOL_LAUNCH(k_gram_rhs, dim3((unsigned)(dp / 64), (unsigned)fs.k),
                     dim3(256), 0, s, X, ldx, Y, ldy, d, c, dp, fs, vec_ok, C,
                     yy);
  if (fs.k <= 8)
    PICHOL_LAUNCH(k_gram_combine_h<8>, dim3((unsigned)tri(nt), 4u), dim3(256),
                  0, s, d, nt, fs, G, H, S);
  else
    PICHOL_LAUNCH(k_gram_combine_h<0>, dim3((unsigned)tri(nt), (unsigned)fs.k),
                  dim3(256), 0, s, d, nt, fs, G, H, S);
  const int64_t nb = dp * c;
  unsigned bx = (unsigned)((nb + 255) / 256);
  if (bx > 2048) bx = 2048;
  PICHOL_LAUNCH(k_gram_combine_b, dim3(bx, (unsigned)fs.k), dim3(256), 0,
                     s, nb, fs, C, B);
  return hipGetLastError();
}

}  // namespace pichol
