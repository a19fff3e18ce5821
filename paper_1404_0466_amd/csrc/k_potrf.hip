// Batched Cholesky factorization of shifted matrices H + lambda I
// (Sec. 3.2; Algorithm 1 step 1 and the exact per-lambda baseline).
//
// Blocked right-looking algorithm on 128-wide panels over the tile-packed
// layout.  For panel kk of every matrix in the batch:
//   1. k_potrf_diag   factors the diagonal tile in LDS and writes the
//                     inverse of the factor to a scratch tile;
//   2. k_potrf_panel  forms the tiles below it as A_{I,kk} L_kk^{-T}
//                     (an FP64 MFMA product with the inverse);
//   3. k_potrf_update subtracts L_{I,kk} L_{J,kk}^T from every trailing tile
//                     (FP64 MFMA, the bulk of the flops).
// One launch of each kernel covers the whole batch, so a batch of B
// matrices of order d fills the GPU with B * (trailing tiles) workgroups.
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace pichol {

// L(m*nshift + s) = H(m) + lam_s I: lower part copied, shift on the first d
// diagonal entries, identity padding, zeros above the diagonal of diagonal
// tiles.  Also clears info.  Matrices m share their shift set in groups of
// lam_group: matrix m uses lam[(m / lam_group) * nshift + s].
__global__ void __launch_bounds__(256) k_shift_copy(int64_t d, int64_t S,
                                                    const double* H,
                                                    int nshift,
                                                    const double* lam,
                                                    int lam_group,
                                                    double* L, int* info) {
  const int64_t ms = blockIdx.y;
  const int64_t m = ms / nshift;
  const int s = (int)(ms % nshift);
  const int I = tri_row(blockIdx.x), J = blockIdx.x - (int)tri(I);
  const double shift = lam[(m / lam_group) * nshift + s];
  const double* h = H + m * S + tile_off(I, J);
  double* l = L + ms * S + tile_off(I, J);
  const int tid = threadIdx.x;
#pragma unroll
  for (int it = 0; it < 16; it += 8) {
    v4d v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ld4(h + ((it + u) * 256 + tid) * 4);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = ((it + u) * 256 + tid) * 4;
      const int64_t j = (int64_t)J * NB + (e >> 7);
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int64_t i = (int64_t)I * NB + ((e + x) & (NB - 1));
        if (i >= d || j >= d)
          v[u][x] = (i == j) ? 1.0 : 0.0;
        else if (i < j)
          v[u][x] = 0.0;
        else if (i == j)
          v[u][x] += shift;
      }
      st4(l + e, v[u]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) info[ms] = 0;
}

// Diagonal tile kk of factor f, in LDS (column-major, a[c*128 + r]):
//  factorization in four 32-column blocks -- the 32 x 32 diagonal block by
//  one wavefront with its rows in registers (readlane broadcasts, no
//  barriers), the rows below it by forward substitution one row per thread,
//  the trailing part by 4 x 4 register-blocked updates;
//  then the inverse of the factor, recursively: the eight 16 x 16 diagonal
//  blocks inverted by half-wavefronts, combined pairwise with
//  [[A,0],[B,C]]^{-1} = [[A^{-1},0],[-C^{-1} B A^{-1}, C^{-1}]].
// Writes the factor tile (zeros above the diagonal) and its inverse to linv.
__global__ void __launch_bounds__(256) k_potrf_diag(int64_t d, int64_t S,
                                                    int kk, double* L,
                                                    int* info, double* linv) {
  __shared__ double a[NB2];
  __shared__ double grp[32 * 4];  // one 4-column group of the 32 x 32 block
  __shared__ double rdiag[NB];    // reciprocals of the factor's diagonal
  const int f = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double* tile = L + (int64_t)f * S + tile_off(kk, kk);
  tile_to_lds(a, tile, tid);
  __syncthreads();

  for (int jb = 0; jb < 4; ++jb) {
    const int j0 = 32 * jb;
    // (1) diagonal 32 x 32 block, wave 0, lane = row j0 + lane.  Columns
    // are factored in groups of four: inside a group by rank-1 updates with
    // readlane broadcasts; then each lane publishes its row of the group in
    // LDS and the trailing columns take the group's four contributions from
    // there (one broadcast read per row instead of four readlane pairs).
    // The subtractions keep the order of plain right-looking elimination.
    if (w == 0) {
      double r[32];
      double myinv = 0.0;  // 1 / L(j0+lane, j0+lane)
#pragma unroll
      for (int k = 0; k < 32; ++k)
        r[k] = (lane < 32 && k <= lane) ? a[(j0 + k) * NB + j0 + lane] : 0.0;
#pragma unroll
      for (int jg = 0; jg < 32; jg += 4) {
#pragma unroll
        for (int j = jg; j < jg + 4; ++j) {
          const double piv = bcast_lane(r[j], j);
          if (lane == 0 && !(piv > 0.0) && info[f] == 0 &&
              (int64_t)kk * NB + j0 + j < d)
            info[f] = kk * NB + j0 + j + 1;
          double ljj, inv;
          sqrt_rsqrt(piv, ljj, inv);
          if (lane == j) {
            r[j] = ljj;
            myinv = inv;
          } else if (lane > j) {
            r[j] = r[j] * inv;
          }
#pragma unroll
          for (int k = j + 1; k < jg + 4; ++k) {
            const double lkj = bcast_lane(r[j], k);
            if (lane >= k) r[k] -= r[j] * lkj;
          }
        }
        if (jg + 4 < 32) {
          if (lane < 32)
            *(v4d*)(grp + 4 * lane) = v4d{r[jg], r[jg + 1], r[jg + 2], r[jg + 3]};
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int k = jg + 4; k < 32; ++k) {
            const v4d lk = *(const v4d*)(grp + 4 * k);
            if (lane >= k) {
              r[k] -= r[jg] * lk[0];
              r[k] -= r[jg + 1] * lk[1];
              r[k] -= r[jg + 2] * lk[2];
              r[k] -= r[jg + 3] * lk[3];
            }
          }
          __builtin_amdgcn_wave_barrier();
        }
      }
      if (lane < 32) {
#pragma unroll
        for (int k = 0; k < 32; ++k)
          if (k <= lane) a[(j0 + k) * NB + j0 + lane] = r[k];
        rdiag[j0 + lane] = myinv;
      }
    }
    __syncthreads();
    if (jb == 3) break;
    // (2) rows below: X = A L_d^{-T}, one row per thread
    const int nrow = NB - j0 - 32;
    if (tid < nrow) {
      const int i = j0 + 32 + tid;
      double x[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) x[k] = a[(j0 + k) * NB + i];
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        x[j] = x[j] * rdiag[j0 + j];
#pragma unroll
        for (int p = j + 1; p < 32; ++p) x[p] -= x[j] * a[(j0 + j) * NB + j0 + p];
      }
#pragma unroll
      for (int k = 0; k < 32; ++k) a[(j0 + k) * NB + i] = x[k];
    }
    __syncthreads();
    // (3) trailing update of rows/columns [j0+32, 128), 4 x 4 blocks
    const int nb4 = nrow / 4;
    const int nblk = nb4 * (nb4 + 1) / 2;
    for (int b = tid; b < nblk; b += blockDim.x) {
      int bi = (int)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
      while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
      while (bi * (bi + 1) / 2 > b) --bi;
      const int bj = b - bi * (bi + 1) / 2;
      const int r0 = j0 + 32 + 4 * bi, c0 = j0 + 32 + 4 * bj;
      double acc[4][4] = {};
#pragma unroll 8
      for (int p = 0; p < 32; ++p) {
        const double* col = a + (j0 + p) * NB;
        double xr[4], xc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          xr[u] = col[r0 + u];
          xc[u] = col[c0 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += xr[u] * xc[v];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (r0 + u >= c0 + v) a[(c0 + v) * NB + r0 + u] -= acc[u][v];
    }
    __syncthreads();
  }

  tile_lower_from_lds(tile, a, tid);

  __syncthreads();
  invert_lower_lds(a, tid, rdiag);
  double* li = linv + (int64_t)f * NB2;
  tile_lower_from_lds(li, a, tid);
}

// Panel tile (I, kk), I > kk: X = A L_kk^{-T}, in place.  The wave computes
// D'(n,m) = sum_p Linv(n,p) A(m,p) = X(m,n), stored at n*128 + m.  Linv is
// lower triangular, so the sum stops at the wave's last n.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_potrf_panel(int64_t S, int kk,
                                                     double* L,
                                                     const double* linv) {
  const int f = blockIdx.y;
  const int I = kk + 1 + blockIdx.x;
  const int w = threadIdx.x >> 6, wi = w >> 1, wj = w & 1;
  double* tile = L + (int64_t)f * S + tile_off(I, kk);
  const double* li = linv + (int64_t)f * NB2;
  Acc64 acc;
  acc.zero();
  mma_panel(acc, li + wi * 64, NB, tile + wj * 64, NB, wi * 64 + 64);
  __syncthreads();  // the whole tile is read before any part is overwritten
  const LaneXY lx;
  const int m0 = wj * 64 + lx.col0();
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const int n = wi * 64 + lx.row(v, bi);
      st4(tile + n * NB + m0, acc.row(v, bi));
    }
}

__device__ inline void mma_any(Acc64& acc, const double* a, int64_t lda,
                               const double* b, int64_t ldb, int K) {
  mma_panel(acc, a, lda, b, ldb, K);
}
__device__ inline void mma_any(Acc64F& acc, const double* a, int64_t lda,
                               const double* b, int64_t ldb, int K) {
  mma_panel_f32(acc, a, lda, b, ldb, K);
}

// Trailing tile (I,J): A_IJ -= sum_{c in [c0,c1)} L_Ic L_Jc^T, for the
// tiles of the triangle j0 <= J <= I (mode 0), of the column J = j0
// (mode 1), or of the two columns J = j0, j0+1 (mode 2).
// The wave computes D'(n,m) = sum_p L_Jc(n,p) L_Ic(m,p) = update(m,n) and
// subtracts it from the tile in its epilogue.  Two workgroups share a CU
// (the register budget is capped for two waves per SIMD), so one's
// read-modify-write epilogue overlaps the other's products.  Logical
// workgroup ids are laid out matrix by matrix and spread over the XCDs in
// contiguous ranges.
template <typename ACC>
__device__ inline void potrf_update_body(int64_t S, int nt, int j0, int mode, int c0, int c1, int ntile,
               double* L) {
  const int id = xcd_remap(blockIdx.x, gridDim.x);
  const int f = id / ntile;
  const int t = id - f * ntile;
  int I, J;
  if (mode == 0) {
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
  if (I == J && wi > wj) return;  // block strictly above the diagonal
  double* Lf = L + (int64_t)f * S;
  double* ct = Lf + tile_off(I, J);
  const LaneXY lx;
  const int m0 = wj * 64 + lx.col0();
  ACC acc;
  acc.zero();
  for (int c = c0; c < c1; ++c)
    mma_any(acc, Lf + tile_off(J, c) + wi * 64, NB,
            Lf + tile_off(I, c) + wj * 64, NB, NB);
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const int n = wi * 64 + ACC::row_of(lx.lq, v, bi);
      double* p = ct + n * NB + m0;
      const v4d val = acc.row(v, bi);
      if (I != J || wi != wj) {
        st4(p, ld4(p) - val);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (m0 + e >= n) p[e] -= val[e];
      }
    }
}

hipError_t launch_shift_copy(int64_t d, int nmat, const double* H, int nshift,
                             const double* lam_dev, int lam_group, double* L,
                             int* info, hipStream_t s) {
  const int64_t nt = ntiles_of(d);
  PICHOL_LAUNCH(k_shift_copy,
                     dim3((unsigned)tri(nt), (unsigned)(nmat * nshift)),
                     dim3(256), 0, s, d, packed_elems_of(d), H, nshift,
                     lam_dev, lam_group, L, info);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_potrf_update(int64_t S, int nt, int j0, int mode, int c0, int c1, int ntile,
               double* L) {
  potrf_update_body<Acc64>(S, nt, j0, mode, c0, c1, ntile, L);
}

// Mixed precision: the same update with the products on FP32 MFMA (operands
// rounded to FP32, FP32 accumulation over the 256-long sums); the tile
// itself stays FP64.  FP32 accumulators take half the registers, so four
// workgroups share a CU (measured faster than two at d = 4096).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_potrf_update_f32(int64_t S, int nt, int j0, int mode, int c0, int c1,
                   int ntile, double* L) {
  potrf_update_body<Acc64F>(S, nt, j0, mode, c0, c1, ntile, L);
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

// Panels are factored in pairs with a delayed update: after panel kk only
// the next panel column is updated, panel kk+1 is factored, and the rest of
// the trailing matrix receives both panels' contributions in one rank-256
// update.  With the look-ahead option on, that update is split: the two
// columns the next pair factors first stay on the caller's stream, the
// remainder runs on a side stream, so the next pair's diagonal
// factorizations and panel solves (short, latency-bound launches) overlap
// the bulk of the update.
hipError_t launch_potrf_blocked(int64_t d, int nfac, double* L, int* info,
                                double* linv_ws, int mixed, int lookahead,
                                int group, hipStream_t s) {
  const int nt = (int)ntiles_of(d);
  const int64_t S = packed_elems_of(d);
  std::unique_lock<std::mutex> lk(g_side_mu, std::defer_lock);
  if (lookahead) lk.lock();
  SideStream* side = lookahead ? side_stream() : nullptr;
  auto diag_panel = [&](int kk) {
    PICHOL_LAUNCH(k_potrf_diag, dim3((unsigned)nfac), dim3(256), 0, s, d, S,
                  kk, L, info, linv_ws);
    const int rest = nt - kk - 1;
    if (rest > 0)
      PICHOL_LAUNCH(k_potrf_panel, dim3((unsigned)rest, (unsigned)nfac),
                    dim3(256), 0, s, S, kk, L, linv_ws);
  };
  auto update = [&](hipStream_t st, int j0, int mode, int c0, int c1) {
    const int rest = nt - j0;
    if (rest <= 0) return;
    const int m = mode == 0 ? 0 : (mode < rest ? mode : rest);
    const int ntile = m == 0 ? (int)tri(rest) : m * rest - m * (m - 1) / 2;
    if (mixed)
      PICHOL_LAUNCH(k_potrf_update_f32, dim3((unsigned)(ntile * nfac)),
                    dim3(256), 0, st, S, nt, j0, m, c0, c1, ntile, L);
    else
      PICHOL_LAUNCH(k_potrf_update, dim3((unsigned)(ntile * nfac)), dim3(256),
                    0, st, S, nt, j0, m, c0, c1, ntile, L);
  };
  const int G = group > 0 ? group : option_panel_group();
  if (!side || G != 2) {
    // Panels in groups of G: before its diagonal factorization, column
    // kk+u receives the group's earlier panels (K = 128 u); after the group,
    // one update of rank 128 G reaches the rest of the trailing matrix.
    for (int kk = 0; kk < nt; kk += G) {
      for (int u = 0; u < G && kk + u < nt; ++u) {
        if (u > 0) update(s, kk + u, 1, kk, kk + u);
        diag_panel(kk + u);
      }
      if (kk + G < nt) update(s, kk + G, 0, kk, kk + G);
    }
    return hipGetLastError();
  }
  int ring = 0;
  bool pending = false;  // a side-stream update not yet joined
  hipEvent_t joined = nullptr;
  for (int kk = 0; kk < nt; kk += 2) {
    diag_panel(kk);
    if (kk + 1 >= nt) break;
    update(s, kk + 1, 1, kk, kk + 1);  // next panel column only
    diag_panel(kk + 1);
    if (kk + 2 >= nt) break;
    // columns kk+2, kk+3 also received the previous pair's remainder
    if (pending) {
      hipStreamWaitEvent(s, joined, 0);
      pending = false;
    }
    if (side && kk + 4 < nt) {
      hipEvent_t ready = side->ev[ring++ & 7];
      hipEventRecord(ready, s);
      update(s, kk + 2, 2, kk, kk + 2);
      hipStreamWaitEvent(side->stream, ready, 0);
      update(side->stream, kk + 4, 0, kk, kk + 2);
      joined = side->ev[ring++ & 7];
      hipEventRecord(joined, side->stream);
      pending = true;
    } else {
      update(s, kk + 2, 0, kk, kk + 2);
    }
  }
  if (pending) hipStreamWaitEvent(s, joined, 0);
  return hipGetLastError();
}

}  // namespace pichol
