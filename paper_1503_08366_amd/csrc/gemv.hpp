// Bandwidth-bound matrix-vector kernels over a dense row-major matrix with a
// 64-element-aligned leading dimension (entries past column n are zero).
//
// gemv_t: column sums  out_r[j] = sum_i op(A_ij) v_r[i]   (A^T v), split over
//         row ranges; each split writes float64 partials, the last split of a
//         column tile reduces them in split order (deterministic) and hands
//         each column to an epilogue.
// gemv_n: row dots     out_r[i] = sum_j op(A_ij) v_r[j]   (A v), LPR lanes per
//         row, the vectors staged in LDS, float64 accumulation.
//
// op is the identity or the elementwise square (for the equilibration sums).
// Matrix elements are read with 16-byte vector loads (4 floats / 2 doubles
// per lane) and widened to float64 before accumulation.
#pragma once

#include "common.hpp"

namespace pogs {

template <bool SQUARE> __device__ inline double elem_op(double a) {
  if constexpr (SQUARE) return a * a;
  else return a;
}

// ---------------------------------------------------------------------------
// gemv_t
// ---------------------------------------------------------------------------
// Epilogue interface (Epi):
//   bool skip() const                      -> exit at once (solver stopped)
//   double column(int j, double s0, double s1) -> per-column finish, j < n;
//                                            returns a value summed per tile
//   void tile_done(int tile, double sum)   -> called by thread 0 of the tile's
//                                            reducing workgroup
//   static constexpr bool kFinal           -> call final() in the last tile
//   void final(double *lds)                -> whole workgroup, after all tiles
template <typename TA, typename TV, int NRHS, bool SQUARE, class Epi>
__global__ __launch_bounds__(kBlock) void gemv_t_kernel(
    const TA *__restrict__ A, int m, int n, int ld, const TV *__restrict__ v0,
    const TV *__restrict__ v1, int rows_per_split, double *__restrict__ part, int ncolp,
    unsigned *tile_cnt, unsigned *fin_cnt, Epi epi) {
  using V = typename Vec16<TA>::type;
  constexpr int VN = Vec16<TA>::N;
  constexpr int TILE = kWave * VN;
  __shared__ double red[4][NRHS][TILE];
  __shared__ double bs[kBlock / kWave];
  __shared__ int flag;
  if (epi.skip()) return;

  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = blockIdx.x;
  const int split = blockIdx.y;
  const int col = tile * TILE + lane * VN;
  const int r0 = split * rows_per_split;
  const int r1 = min(m, r0 + rows_per_split);

  double acc[NRHS][VN];
#pragma unroll
  for (int r = 0; r < NRHS; ++r)
#pragma unroll
    for (int c = 0; c < VN; ++c) acc[r][c] = 0.0;

  if (col < n) {
    const TA *base = A + col;
    int i = r0 + w;
    for (; i + 12 < r1; i += 16) {
      V a[4];
      double s[4][NRHS];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = *reinterpret_cast<const V *>(base + (size_t)(i + 4 * u) * ld);
        s[u][0] = (double)v0[i + 4 * u];
        if constexpr (NRHS > 1) s[u][1] = (double)v1[i + 4 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < VN; ++c) {
          const double e = elem_op<SQUARE>((double)a[u][c]);
#pragma unroll
          for (int r = 0; r < NRHS; ++r) acc[r][c] = fma(e, s[u][r], acc[r][c]);
        }
    }
    for (; i < r1; i += 4) {
      const V a = *reinterpret_cast<const V *>(base + (size_t)i * ld);
      double s[NRHS];
      s[0] = (double)v0[i];
      if constexpr (NRHS > 1) s[1] = (double)v1[i];
#pragma unroll
      for (int c = 0; c < VN; ++c) {
        const double e = elem_op<SQUARE>((double)a[c]);
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc[r][c] = fma(e, s[r], acc[r][c]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NRHS; ++r)
#pragma unroll
    for (int c = 0; c < VN; ++c) red[w][r][lane * VN + c] = acc[r][c];
  __syncthreads();
  if (threadIdx.x < TILE) {
    const int t = threadIdx.x;
    const int cg = tile * TILE + t;
#pragma unroll
    for (int r = 0; r < NRHS; ++r) {
      const double v = (red[0][r][t] + red[1][r][t]) + (red[2][r][t] + red[3][r][t]);
      part[(size_t)(split * NRHS + r) * ncolp + cg] = v;
    }
  }
  if (!arrive_last(&tile_cnt[tile], gridDim.y, &flag)) return;

  // Last split of this tile: reduce the partials in split order.
  double contrib = 0.0;
  if (threadIdx.x < TILE) {
    const int cg = tile * TILE + threadIdx.x;
    double s[2] = {0.0, 0.0};
    for (int sp = 0; sp < (int)gridDim.y; ++sp)
#pragma unroll
      for (int r = 0; r < NRHS; ++r) s[r] += load_agent(part + (size_t)(sp * NRHS + r) * ncolp + cg);
    if (cg < n) contrib = epi.column(cg, s[0], s[1]);
  }
  const double tsum = block_sum(contrib, bs);
  if (threadIdx.x == 0) epi.tile_done(tile, tsum);
  if constexpr (Epi::kFinal) {
    if (arrive_last(fin_cnt, gridDim.x, &flag)) epi.final(bs);
  }
}

// ---------------------------------------------------------------------------
// gemv_n
// ---------------------------------------------------------------------------
// Epilogue interface:
//   bool skip() const
//   double row(int i, double s0, double s1)  -> per-row finish (i < m); value
//                                             summed per workgroup
//   void block_done(int block, double sum)   -> thread 0 of each workgroup
//   static constexpr bool kFinal; void final(double *lds)
template <typename TV> struct GemvNChunk { static constexpr int value = 8192 / sizeof(TV) * 2; };

template <typename TA, typename TV, int NRHS, bool SQUARE, int LPR, int RPT, class Epi>
__global__ __launch_bounds__(kBlock) void gemv_n_kernel(
    const TA *__restrict__ A, int m, int n, int ld, const TV *__restrict__ v0,
    const TV *__restrict__ v1, unsigned *cnt, Epi epi) {
  using V = typename Vec16<TA>::type;
  constexpr int VN = Vec16<TA>::N;
  constexpr int CH = GemvNChunk<TV>::value;  // vector elements staged per chunk
  constexpr int GPW = kWave / LPR;            // row groups per wave
  constexpr int ROWS = (kBlock / kWave) * GPW * RPT;
  __shared__ TV vs[NRHS][CH];
  __shared__ double bs[kBlock / kWave];
  __shared__ int flag;
  if (epi.skip()) return;

  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x >> 6;
  const int sub = lane % LPR;
  const int grp = lane / LPR;
  const int row_base = blockIdx.x * ROWS + (w * GPW + grp) * RPT;

  double acc[RPT][NRHS];
#pragma unroll
  for (int t = 0; t < RPT; ++t)
#pragma unroll
    for (int r = 0; r < NRHS; ++r) acc[t][r] = 0.0;

  for (int c0 = 0; c0 < n; c0 += CH) {
    const int clen = min(CH, ld - c0);  // multiple of 64, inside the row
    __syncthreads();
    for (int t = threadIdx.x; t < clen; t += kBlock) {
      const int j = c0 + t;
      vs[0][t] = j < n ? v0[j] : TV(0);
      if constexpr (NRHS > 1) vs[1][t] = j < n ? v1[j] : TV(0);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int i = row_base + t;
      if (i < m) {
        const TA *rowp = A + (size_t)i * ld + c0;
        int c = sub * VN;
        for (; c + 3 * LPR * VN < clen; c += 4 * LPR * VN) {
          V a[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) a[u] = *reinterpret_cast<const V *>(rowp + c + u * LPR * VN);
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < VN; ++k) {
              const double e = elem_op<SQUARE>((double)a[u][k]);
              acc[t][0] = fma(e, (double)vs[0][c + u * LPR * VN + k], acc[t][0]);
              if constexpr (NRHS > 1) acc[t][1] = fma(e, (double)vs[1][c + u * LPR * VN + k], acc[t][1]);
            }
        }
        for (; c < clen; c += LPR * VN) {
          const V a = *reinterpret_cast<const V *>(rowp + c);
#pragma unroll
          for (int k = 0; k < VN; ++k) {
            const double e = elem_op<SQUARE>((double)a[k]);
            acc[t][0] = fma(e, (double)vs[0][c + k], acc[t][0]);
            if constexpr (NRHS > 1) acc[t][1] = fma(e, (double)vs[1][c + k], acc[t][1]);
          }
        }
      }
    }
  }
  double contrib = 0.0;
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    double s0 = group_sum<LPR>(acc[t][0]);
    double s1 = 0.0;
    if constexpr (NRHS > 1) s1 = group_sum<LPR>(acc[t][1]);
    const int i = row_base + t;
    if (sub == 0 && i < m) contrib += epi.row(i, s0, s1);
  }
  const double bsum = block_sum(contrib, bs);
  if (threadIdx.x == 0) epi.block_done(blockIdx.x, bsum);
  if constexpr (Epi::kFinal) {
    if (arrive_last(cnt, gridDim.x, &flag)) epi.final(bs);
  }
}

template <int LPR, int RPT> constexpr int gemv_n_rows_per_block() {
  return (kBlock / kWave) * (kWave / LPR) * RPT;
}

}  // namespace pogs
