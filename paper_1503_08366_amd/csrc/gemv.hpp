// Bandwidth-bound matrix-vector kernels over a dense row-major matrix with a
// 64-element-aligned leading dimension (entries past column n are zero).
//
// gemv_t: column sums  out_r[j] = sum_i op(A_ij) v_r[i]   (A^T v), split over
//         row ranges; each split writes float64 partials.  A second, small
//         kernel (gemv_t_finish) sums the partials in split order
//         (deterministic) and hands each column to an epilogue.  The split
//         is a kernel boundary rather than a "last workgroup" handshake: on
//         gfx950 a device-scope fence writes back and invalidates the whole
//         L2, which costs far more per workgroup than one extra launch.
// gemv_n: row dots     out_r[i] = sum_j op(A_ij) v_r[j]   (A v), LPR lanes per
//         row, the vectors staged in LDS, float64 accumulation.
//
// op is the identity or the elementwise square (for the equilibration sums).
// Matrix elements are read with 16-byte vector loads (4 floats / 2 doubles
// per lane) and widened to float64 before accumulation.
#pragma once

#include <cstdint>
#include <utility>

#include "common.hpp"

namespace pogs {

// Loads of the matrix.  NT (non-temporal) for a matrix larger than the
// last-level cache, which each pass streams once: it then does not displace
// the vectors and partial sums (measured on gfx950: 100000 x 1000 row pass
// 73 -> 64 us).  A matrix that fits is loaded normally and partly stays cached
// from one pass to the next (20000 x 2000: the iteration is 3 us faster so).
template <bool NT, typename V> __device__ __forceinline__ V mat_load(const V *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool SQUARE> __device__ inline double elem_op(double a) {
  if constexpr (SQUARE) return a * a;
  else return a;
}

// ---------------------------------------------------------------------------
// gemv_t
// ---------------------------------------------------------------------------
// Epilogue interface (Epi):
//   bool skip() const                          -> exit at once (solver stopped)
//   double column(int j, double s0, double s1) -> per-column finish, j < n;
//                                                returns a value summed per tile
//   void tile_done(int tile, double sum)       -> thread 0 of the tile's workgroup
// The finish kernel also accepts column() returning Sum2 (two values summed
// per tile) with tile_done(int tile, double sum_a, double sum_b).
template <typename TA, typename TV, int NRHS, bool SQUARE, class Epi, bool NT = false>
__device__ __forceinline__ void gemv_t_body(
    const Blk &b, const TA *__restrict__ A, int m, int n, int ld, const TV *__restrict__ v0,
    const TV *__restrict__ v1, int rows_per_split, double *__restrict__ part, int ncolp, const Epi &epi) {
  using V = typename Vec16<TA>::type;
  constexpr int VN = Vec16<TA>::N;
  constexpr int TILE = kWave * VN;
  __shared__ double red[4][NRHS][TILE];
  const bool stopped = epi.skip();  // used once the first group's loads are out

  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = b.x;
  const int split = b.y;
  const int col = tile * TILE + lane * VN;
  const int r0 = split * rows_per_split;
  const int r1 = min(m, r0 + rows_per_split);

  double acc[NRHS][VN];
#pragma unroll
  for (int r = 0; r < NRHS; ++r)
#pragma unroll
    for (int c = 0; c < VN; ++c) acc[r][c] = 0.0;

  // groups of 8 of the wave's rows (4 apart), loaded together, then used
  const TA *base = A + (col < n ? col : 0);
  V a[8];
  double s[8][NRHS];
  auto group_load = [&](int i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = mat_load<NT>(reinterpret_cast<const V *>(base + (size_t)(i + 4 * u) * ld));
      s[u][0] = (double)v0[i + 4 * u];
      if constexpr (NRHS > 1) s[u][1] = (double)v1[i + 4 * u];
    }
  };
  auto group_fma = [&]() {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < VN; ++c) {
        const double e = elem_op<SQUARE>((double)a[u][c]);
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc[r][c] = fma(e, s[u][r], acc[r][c]);
      }
  };
  const bool first = col < n && r0 + w + 28 < r1;
  if (first) group_load(r0 + w);
  if (stopped) return;

  if (col < n) {
    int i = r0 + w;
    if (first) {
      group_fma();
      i += 32;
    }
    for (; i + 28 < r1; i += 32) {
      group_load(i);
      group_fma();
    }
    for (; i < r1; i += 4) {
      const V x = mat_load<NT>(reinterpret_cast<const V *>(base + (size_t)i * ld));
      double sv[NRHS];
      sv[0] = (double)v0[i];
      if constexpr (NRHS > 1) sv[1] = (double)v1[i];
#pragma unroll
      for (int c = 0; c < VN; ++c) {
        const double e = elem_op<SQUARE>((double)x[c]);
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc[r][c] = fma(e, sv[r], acc[r][c]);
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
}

template <typename TA, typename TV, int NRHS, bool SQUARE, class Epi, bool NT = false>
__global__ __launch_bounds__(kBlock) void gemv_t_kernel(const TA *__restrict__ A, int m, int n, int ld,
                                                        const TV *__restrict__ v0, const TV *__restrict__ v1,
                                                        int rows_per_split, double *__restrict__ part, int ncolp,
                                                        Epi epi) {
  gemv_t_body<TA, TV, NRHS, SQUARE, Epi, NT>(hw_block(), A, m, n, ld, v0, v1, rows_per_split, part, ncolp, epi);
}

// Sum the split partials of kFinishCols columns (block b.x): the threads
// form kBlock / kFinishCols split groups, group g sums the splits g,
// g + groups, ...; the group sums are then added in group order (a fixed
// order, so results are deterministic); each column is finished by the
// epilogue and the block's sum goes to tile_done(b.x, .).
template <int NRHS, class Epi>
__device__ __forceinline__ void gemv_t_finish_body(const Blk &b, int n, int splits, const double *__restrict__ part,
                                                   int ncolp, const Epi &epi) {
  constexpr int G = kBlock / kFinishCols;
  __shared__ double red[G][2][kFinishCols];
  __shared__ double bs[kBlock / kWave];
  const bool stopped = epi.skip();  // used once the partial loads are out
  const int c = threadIdx.x % kFinishCols;
  const int g = threadIdx.x / kFinishCols;
  const int cg = b.x * kFinishCols + c;
  double s[2] = {0.0, 0.0};
  if (cg < ncolp) {
#pragma unroll 4
    for (int sp = g; sp < splits; sp += G)
#pragma unroll
      for (int r = 0; r < NRHS; ++r) s[r] += part[(size_t)(sp * NRHS + r) * ncolp + cg];
  }
  if (stopped) return;
  red[g][0][c] = s[0];
  red[g][1][c] = s[1];
  __syncthreads();
  using R = decltype(epi.column(0, 0.0, 0.0));
  R contrib{};
  if (g == 0 && cg < n) {
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      t0 += red[k][0][c];
      t1 += red[k][1][c];
    }
    contrib = epi.column(cg, t0, t1);
  }
  if constexpr (std::is_same<R, Sum2>::value) {
    const double ta = block_sum(contrib.a, bs);
    const double tb = block_sum(contrib.b, bs);
    if (threadIdx.x == 0) epi.tile_done(b.x, ta, tb);
  } else {
    const double tsum = block_sum(contrib, bs);
    if (threadIdx.x == 0) epi.tile_done(b.x, tsum);
  }
}

template <int NRHS, class Epi>
__global__ __launch_bounds__(kBlock) void gemv_t_finish_kernel(int n, int splits, const double *__restrict__ part,
                                                                int ncolp, Epi epi) {
  gemv_t_finish_body<NRHS, Epi>(hw_block(), n, splits, part, ncolp, epi);
}

// ---------------------------------------------------------------------------
// gemv_n
// ---------------------------------------------------------------------------
// Epilogue interface:
//   bool skip() const
//   double row(int i, double s0, double s1)  -> per-row finish (i < m); value
//                                             summed per workgroup
//   void block_done(int block, double sum)   -> thread 0 of each workgroup
template <typename TV> struct GemvNChunk { static constexpr int value = 8192 / sizeof(TV) * 2; };

template <typename TA, typename TV, int NRHS, bool SQUARE, int LPR, int RPT, class Epi, bool NT = false>
__device__ __forceinline__ void gemv_n_body(
    const Blk &b, const TA *__restrict__ A, int m, int n, int ld, const TV *__restrict__ v0,
    const TV *__restrict__ v1, const Epi &epi) {
  using V = typename Vec16<TA>::type;
  constexpr int VN = Vec16<TA>::N;
  constexpr int CH = GemvNChunk<TV>::value;  // vector elements staged per chunk
  constexpr int GPW = kWave / LPR;            // row groups per wave
  constexpr int ROWS = (kBlock / kWave) * GPW * RPT;
  __shared__ TV vs[NRHS][CH];
  __shared__ double bs[kBlock / kWave];
  if (epi.skip()) return;

  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x >> 6;
  const int sub = lane % LPR;
  const int grp = lane / LPR;
  const int row_base = b.x * ROWS + (w * GPW + grp) * RPT;

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
    // RPT rows side by side, two column steps per trip: up to 2 * RPT
    // independent 16-byte loads in flight per lane.  Rows past m read row
    // m - 1 (valid memory) and are discarded.
    const TA *rowp[RPT];
#pragma unroll
    for (int t = 0; t < RPT; ++t) rowp[t] = A + (size_t)min(row_base + t, m - 1) * ld + c0;
    constexpr int STEP = LPR * VN;
    int c = sub * VN;
    for (; c + STEP < clen; c += 2 * STEP) {
      V a[2][RPT];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int t = 0; t < RPT; ++t) a[u][t] = mat_load<NT>(reinterpret_cast<const V *>(rowp[t] + c + u * STEP));
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int k = 0; k < VN; ++k) {
          const double x0 = (double)vs[0][c + u * STEP + k];
          double x1 = 0.0;
          if constexpr (NRHS > 1) x1 = (double)vs[1][c + u * STEP + k];
#pragma unroll
          for (int t = 0; t < RPT; ++t) {
            const double e = elem_op<SQUARE>((double)a[u][t][k]);
            acc[t][0] = fma(e, x0, acc[t][0]);
            if constexpr (NRHS > 1) acc[t][1] = fma(e, x1, acc[t][1]);
          }
        }
    }
    if (c < clen) {
      V a[RPT];
#pragma unroll
      for (int t = 0; t < RPT; ++t) a[t] = mat_load<NT>(reinterpret_cast<const V *>(rowp[t] + c));
#pragma unroll
      for (int k = 0; k < VN; ++k) {
        const double x0 = (double)vs[0][c + k];
        double x1 = 0.0;
        if constexpr (NRHS > 1) x1 = (double)vs[1][c + k];
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
          const double e = elem_op<SQUARE>((double)a[t][k]);
          acc[t][0] = fma(e, x0, acc[t][0]);
          if constexpr (NRHS > 1) acc[t][1] = fma(e, x1, acc[t][1]);
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
  if (threadIdx.x == 0) epi.block_done(b.x, bsum);
}

template <typename TA, typename TV, int NRHS, bool SQUARE, int LPR, int RPT, class Epi, bool NT = false>
__global__ __launch_bounds__(kBlock) void gemv_n_kernel(const TA *__restrict__ A, int m, int n, int ld,
                                                        const TV *__restrict__ v0, const TV *__restrict__ v1,
                                                        Epi epi) {
  gemv_n_body<TA, TV, NRHS, SQUARE, LPR, RPT, Epi, NT>(hw_block(), A, m, n, ld, v0, v1, epi);
}

// ---------------------------------------------------------------------------
// gemv_n, whole rows per wave (float32 A, rows of at most 256 NC elements)
// ---------------------------------------------------------------------------
// Each wave takes rows gw, gw + W, gw + 2W, ... (W = waves in the grid, gw
// its global index).  A wave loads a whole row with NC 16-byte loads per lane
// (lane l holds columns 4 l + 256 u), multiplies it by the vectors, which the
// workgroup staged once in LDS (float32, the same columns for every row), and
// reduces across the wave.  Two rows are in flight per wave: the loads of
// row r + W are issued before row r is reduced.
//
// Latency is what this pass has to hide, so:
//  - every thread issues its loads of the vectors (16 bytes each where the
//    vector is aligned) before anything else, then the loads of the wave's
//    first row, and only then writes the vectors to LDS and waits at the
//    barrier: the three memory round trips overlap instead of following one
//    another;
//  - the loads of a row are unconditional (a lane whose columns lie past ld
//    reads the row's last 16 bytes again and multiplies them by the zeros
//    staged there), and the row loop branches only on wave-uniform counts,
//    so the compiler waits for exactly the row it is about to use;
//  - the epilogue runs once per 64 rows for all of them: lane t keeps the
//    sums of the batch's row t, and after the batch every lane finishes its
//    row (with the epilogue's own loads issued by all lanes at once) instead
//    of lane 0 finishing each row between two loads.
// Rows of a batch are summed per lane and the block's sum follows the fixed
// order of block_sum, so results do not depend on timing.
template <int NRHS, int NC, class Epi, bool NT = false>
__device__ __forceinline__ void gemv_n_rows_body(const Blk &b, const float *__restrict__ A, int m, int n, int ld,
                                                 const float *__restrict__ v0, const float *__restrict__ v1,
                                                 const Epi &epi) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int CH = 64 * NC;                       // 16-byte pieces of each staged vector
  constexpr int CPT = (CH + kBlock - 1) / kBlock;   // pieces per thread
  __shared__ float xs[NRHS][256 * NC];
  __shared__ double bs[kBlock / kWave];
  const bool stopped = epi.skip();  // used once the first loads are out
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  const int W = b.nx * (kBlock / kWave);
  const int gw = b.x * (kBlock / kWave) + w;

  f4 st[NRHS][CPT];
  const bool aligned = (((uintptr_t)v0 | (uintptr_t)v1) & 15) == 0;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int q = threadIdx.x + kBlock * j;
    const int idx = 4 * q;
    if (q < CH) {
      if (aligned && idx + 3 < n) {
        st[0][j] = *reinterpret_cast<const f4 *>(v0 + idx);
        if constexpr (NRHS > 1) st[1][j] = *reinterpret_cast<const f4 *>(v1 + idx);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          st[0][j][k] = idx + k < n ? v0[idx + k] : 0.f;
          if constexpr (NRHS > 1) st[1][j][k] = idx + k < n ? v1[idx + k] : 0.f;
        }
      }
    }
  }

  const int nrows = gw < m ? (m - 1 - gw) / W + 1 : 0;
  int cofs[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) cofs[u] = min(4 * lane + 256 * u, ld - 4);
  auto load = [&](f4 *dst, int r) {
    const float *rp = A + (size_t)r * ld;
#pragma unroll
    for (int u = 0; u < NC; ++u) dst[u] = mat_load<NT>(reinterpret_cast<const f4 *>(rp + cofs[u]));
  };
  f4 a0[NC], a1[NC];
  if (nrows > 0) load(a0, gw);
  if (stopped) return;  // nothing is written once the solver has stopped

#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int q = threadIdx.x + kBlock * j;
    if (q < CH) {
      *reinterpret_cast<f4 *>(&xs[0][4 * q]) = st[0][j];
      if constexpr (NRHS > 1) *reinterpret_cast<f4 *>(&xs[1][4 * q]) = st[1][j];
    }
  }
  __syncthreads();

  double contrib = 0.0;
  double k0 = 0.0, k1 = 0.0;
  auto compute = [&](const f4 *a, int slot) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const f4 x0 = *reinterpret_cast<const f4 *>(&xs[0][4 * lane + 256 * u]);
      f4 x1;
      if constexpr (NRHS > 1) x1 = *reinterpret_cast<const f4 *>(&xs[1][4 * lane + 256 * u]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double e = (double)a[u][k];
        s0 = fma(e, (double)x0[k], s0);
        if constexpr (NRHS > 1) s1 = fma(e, (double)x1[k], s1);
      }
    }
    s0 = wave_sum(s0);
    if constexpr (NRHS > 1) s1 = wave_sum(s1);
    if (lane == slot) {
      k0 = s0;
      k1 = s1;
    }
  };
  // rows i0 .. i0 + cnt - 1 of the wave per batch (cnt <= 64, even except at
  // the end, so row i is in a0 for even i and in a1 for odd i)
  for (int i0 = 0; i0 < nrows; i0 += kWave) {
    const int cnt = min(kWave, nrows - i0);
    for (int t = 0; t < cnt; t += 2) {
      const int i = i0 + t;
      if (i + 1 < nrows) load(a1, gw + (i + 1) * W);
      compute(a0, t);
      if (t + 1 >= cnt) break;
      if (i + 2 < nrows) load(a0, gw + (i + 2) * W);
      compute(a1, t + 1);
    }
    if (lane < cnt) contrib += epi.row(gw + (i0 + lane) * W, k0, k1);
  }
  const double bsum = block_sum(contrib, bs);
  if (threadIdx.x == 0) epi.block_done(b.x, bsum);
}

template <int NRHS, int NC, class Epi, bool NT = false>
__global__ __launch_bounds__(kBlock) void gemv_n_rows_kernel(const float *__restrict__ A, int m, int n, int ld,
                                                             const float *__restrict__ v0,
                                                             const float *__restrict__ v1, Epi epi) {
  gemv_n_rows_body<NRHS, NC, Epi, NT>(hw_block(), A, m, n, ld, v0, v1, epi);
}

template <int LPR, int RPT> constexpr int gemv_n_rows_per_block() {
  return (kBlock / kWave) * (kWave / LPR) * RPT;
}

}  // namespace pogs
