// One-time setup per matrix, on gfx950:
//   layout      : host/device A (f32/f64, row/col-major) -> row-major T, ld % 64 == 0
//   equilibrate : Algorithm 2 (regularised Sinkhorn-Knopp, p = 2,
//                 gamma = (m + n) sqrt(eps_cmp)) for a fixed sweep count, then
//                 the Frobenius normalisation of Section 4.1.2 and A <- D A E
//   gram        : G = A^T A (m >= n) or A A^T (m < n) on MFMA (f32 MFMA with
//                 f32 accumulation inside a K split; splits summed in f64),
//                 K = I + G in float64 (Section 3.5)
//   factor      : blocked Cholesky K = L L^T in float64 (64 x 64 blocks, f64
//                 MFMA for the block products), L^{-1} by blocked substitution
//                 and K^{-1} = L^{-T} L^{-1} accumulated row by row of L^{-1}
//                 in the same steps, stored in T for the iterations.
#include <atomic>

#include "setup.hpp"

namespace pogs {

// ---------------------------------------------------------------------------
// Layout conversion
// ---------------------------------------------------------------------------

template <typename T, typename S>
__global__ __launch_bounds__(256) void layout_kernel(const S *src, int colmajor, int64_t lda, int m,
                                                     int n, T *dst, int ld, unsigned *bad) {
  layout_body<T, S>(hw_block(), src, colmajor, lda, m, n, dst, ld, bad);
}

__global__ __launch_bounds__(256) void layout_rows_f32_kernel(const float *src, int64_t lda, int m, int n,
                                                              float *dst, int ld, unsigned *bad) {
  layout_rows_f32_body(hw_block(), src, lda, m, n, dst, ld, bad);
}

__global__ __launch_bounds__(256) void scale_rows_f32_kernel(float *A, int m, int n, int ld, const double *D,
                                                             const double *E) {
  scale_rows_f32_body(hw_block(), A, m, n, ld, D, E);
}

// Rows per launch column of the 16-byte row kernels: enough workgroups to
// fill the GPU several times over, each thread with a few rows of work.
static int row_blocks(int m) { return std::max(1, std::min(m, 2048)); }

template <typename T>
void launch_layout(const void *src, pogs_dtype sdt, pogs_order ord, int64_t lda, int m, int n, T *dst,
                   int ld, unsigned *bad, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (sdt == POGS_F32 && ord == POGS_ROW_MAJOR && lda % 4 == 0 && ((uintptr_t)src & 15) == 0) {
      hipLaunchKernelGGL(layout_rows_f32_kernel, dim3(cdiv(ld, 1024), row_blocks(m)), dim3(256), 0, s,
                         (const float *)src, lda, m, n, (float *)dst, ld, bad);
      return;
    }
  }
  dim3 grid(cdiv(ld, 32), cdiv(m, 32));
  const int cm = ord == POGS_COL_MAJOR;
  if (sdt == POGS_F32)
    hipLaunchKernelGGL((layout_kernel<T, float>), grid, dim3(256), 0, s, (const float *)src, cm, lda, m,
                       n, dst, ld, bad);
  else
    hipLaunchKernelGGL((layout_kernel<T, double>), grid, dim3(256), 0, s, (const double *)src, cm, lda,
                       m, n, dst, ld, bad);
}

// ---------------------------------------------------------------------------
// Equilibration (Algorithm 2, p = 2) and Frobenius normalisation
// ---------------------------------------------------------------------------


template <int U, int R>
__global__ __launch_bounds__(kBlock) void equil_sweep_kernel(const float *__restrict__ A, int m, int n, int ld,
                                                             int rps, const double *__restrict__ e,
                                                             double *__restrict__ d, double *__restrict__ part,
                                                             int ncolp, double nf, double gamma_m) {
  equil_sweep_body<U, R>(hw_block(), A, m, n, ld, rps, e, d, part, ncolp, nf, gamma_m);
}

__global__ void fill_kernel(double *p, double v, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = v;
}


__global__ __launch_bounds__(256) void equil_finish_kernel(const double *d, const double *e, const double *slots,
                                                           int ntiles, int m, int n, int q, double *D, double *E) {
  equil_finish_body(hw_block(), d, e, slots, ntiles, m, n, q, D, E);
}


template <typename T>
__global__ __launch_bounds__(256) void scale_matrix_kernel(T *A, int m, int n, int ld, const double *D,
                                                           const double *E) {
  scale_matrix_body<T>(hw_block(), A, m, n, ld, D, E);
}

// Workgroups of `kernel` (block threads per workgroup, static LDS only)
// resident on the whole device at once.
int resident_workgroups(const void *kernel, int block) {
  int nb = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, 0) != hipSuccess) nb = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  return std::max(1, nb) * std::max(1, cus);
}

size_t equil_workspace_bytes(int m, int n) {
  int splits, rps, ncolp;
  gemv_t_geometry(m, n, 4, &splits, &rps, &ncolp);
  int s2, r2, nc2;
  gemv_t_geometry(m, n, 8, &s2, &r2, &nc2);
  // the fused float32 sweep writes up to 1024 workgroups of column sums
  const size_t part = std::max<size_t>((size_t)std::max(splits * ncolp, s2 * nc2), (size_t)1024 * ncolp);
  // d, e, colsum, slots, fro2, partials
  return ((size_t)m + 2 * (size_t)n + (size_t)ncolp + 8 + part) * sizeof(double);
}

template <typename T>
int run_equilibrate(T *A, int m, int n, int ld, int iters, double eps_cmp, double *D, double *E, double *ws,
                    size_t ws_bytes, unsigned *counters, hipStream_t s) {
  if (iters <= 0) {
    hipLaunchKernelGGL(fill_kernel, dim3(cdiv(m, 256)), dim3(256), 0, s, D, 1.0, m);
    hipLaunchKernelGGL(fill_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, E, 1.0, n);
    return POGS_OK;
  }
  int splits, rps, ncolp;
  gemv_t_geometry(m, n, sizeof(T), &splits, &rps, &ncolp);
  EqArgs a;
  a.d = ws;
  a.e = a.d + m;
  a.colsum = a.e + n;
  a.slots = a.colsum + n;
  a.fro2 = a.slots + ncolp;
  double *part = a.fro2 + 8;
  if ((size_t)((part + (size_t)splits * ncolp) - ws) * sizeof(double) > ws_bytes) return POGS_ENOMEM;
  const double gamma = (double)(m + n) * sqrt(eps_cmp);
  a.gamma_m = gamma / m;
  a.gamma_n = gamma / n;
  a.mf = m;
  a.nf = n;
  hipLaunchKernelGGL(fill_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, a.e, 1.0, n);
  const int tiles = (int)cdiv(n, gemv_t_tile(sizeof(T)));
  (void)counters;
  if (sizeof(T) == 4 && n <= 4096) {
    // fused sweeps: one pass over A per sweep, as many workgroups as are
    // resident at once (no tail round)
    constexpr int R = 4;
    const int U = (int)cdiv(n, 1024);
    const void *kern = U == 1   ? (const void *)equil_sweep_kernel<1, R>
                       : U == 2 ? (const void *)equil_sweep_kernel<2, R>
                       : U == 3 ? (const void *)equil_sweep_kernel<3, R>
                                : (const void *)equil_sweep_kernel<4, R>;
    const int nwg = (int)std::min<int64_t>(std::min(1024, resident_workgroups(kern, kBlock)), cdiv(m, R));
    const int rps = (int)round_up(cdiv(m, nwg), R);
    const int nsplit = (int)cdiv(m, rps);
    if ((size_t)((part + (size_t)nsplit * ncolp) - ws) * sizeof(double) > ws_bytes) return POGS_ENOMEM;
    for (int it = 0; it < iters; ++it) {
      const float *Af = (const float *)A;
      switch (U) {
        case 1:
          hipLaunchKernelGGL((equil_sweep_kernel<1, R>), dim3(nsplit), dim3(kBlock), 0, s, Af, m, n, ld, rps, a.e,
                             a.d, part, ncolp, a.nf, a.gamma_m);
          break;
        case 2:
          hipLaunchKernelGGL((equil_sweep_kernel<2, R>), dim3(nsplit), dim3(kBlock), 0, s, Af, m, n, ld, rps, a.e,
                             a.d, part, ncolp, a.nf, a.gamma_m);
          break;
        case 3:
          hipLaunchKernelGGL((equil_sweep_kernel<3, R>), dim3(nsplit), dim3(kBlock), 0, s, Af, m, n, ld, rps, a.e,
                             a.d, part, ncolp, a.nf, a.gamma_m);
          break;
        default:
          hipLaunchKernelGGL((equil_sweep_kernel<4, R>), dim3(nsplit), dim3(kBlock), 0, s, Af, m, n, ld, rps, a.e,
                             a.d, part, ncolp, a.nf, a.gamma_m);
          break;
      }
      EpiEqCol ec{a};
      hipLaunchKernelGGL((gemv_t_finish_kernel<1, EpiEqCol>), dim3(cdiv(n, kFinishCols)), dim3(kBlock), 0, s, n,
                         nsplit, (const double *)part, ncolp, ec);
    }
  }
  for (int it = 0; it < iters && !(sizeof(T) == 4 && n <= 4096); ++it) {
    // rows: d = n / (|A|^2 e + gamma/m)
    {
      EpiEqRow er{a};
      constexpr int VN = Vec16<T>::N;
      if (cdiv(n, VN) >= 128)
        hipLaunchKernelGGL((gemv_n_kernel<T, double, 1, true, 64, 1, EpiEqRow>),
                           dim3(cdiv(m, gemv_n_rows_per_block<64, 1>())), dim3(kBlock), 0, s, A, m, n, ld, a.e, a.e,
                           er);
      else
        hipLaunchKernelGGL((gemv_n_kernel<T, double, 1, true, 16, 1, EpiEqRow>),
                           dim3(cdiv(m, gemv_n_rows_per_block<16, 1>())), dim3(kBlock), 0, s, A, m, n, ld, a.e, a.e,
                           er);
    }
    // columns: e = m / (|A^T|^2 d + gamma/n)
    {
      EpiEqCol ec{a};
      hipLaunchKernelGGL((gemv_t_kernel<T, double, 1, true, EpiEqCol>), dim3(tiles, splits), dim3(kBlock), 0, s, A,
                         m, n, ld, a.d, a.d, rps, part, ncolp, ec);
      hipLaunchKernelGGL((gemv_t_finish_kernel<1, EpiEqCol>), dim3(cdiv(n, kFinishCols)), dim3(kBlock), 0, s, n,
                         splits, (const double *)part, ncolp, ec);
    }
  }
  const int q = std::min(m, n);
  hipLaunchKernelGGL(equil_finish_kernel, dim3(cdiv(m + n, 256)), dim3(256), 0, s, a.d, a.e, a.slots,
                     (int)cdiv(n, kFinishCols), m, n, q, D, E);
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL(scale_rows_f32_kernel, dim3(cdiv(n, 1024), row_blocks(m)), dim3(256), 0, s, (float *)A, m, n,
                       ld, D, E);
  else
    hipLaunchKernelGGL((scale_matrix_kernel<T>), dim3(cdiv(n, 256), std::min(m, 32768)), dim3(256), 0, s, A, m, n,
                       ld, D, E);
  return POGS_OK;
}

// ---------------------------------------------------------------------------
// Gram matrix on MFMA
// ---------------------------------------------------------------------------
// G tile (ti, tj) partial over the K range of split blockIdx.y (f32 MFMA).
template <bool TALL>
__global__ __launch_bounds__(256, 4) void gram_f32_kernel(const float *__restrict__ A, int m, int n, int ld,
                                                       int kchunk, int ntp, float *__restrict__ part) {
  __shared__ GramStage st[2];
  int ti, tj;
  tri_index(blockIdx.x, &ti, &tj);
  const int kdim = TALL ? m : n;
  const int k0 = blockIdx.y * kchunk;
  const int k1 = min(kdim, k0 + kchunk);
  float *out = part + ((size_t)blockIdx.y * ntp + blockIdx.x) * kGramTB * kGramTB;
  gram_tile_f32<TALL>(A, m, n, ld, ti, tj, k0, k1, st,
                      [&](int r, int c, float v) { out[r * kGramTB + c] = v; });
}

// Tall float32 matrices: the same tiles and splits from bf16 MFMAs at float32
// accuracy (gram_tile_bf16x6).
__global__ __launch_bounds__(512, 2) void gram_bf16x6_kernel(const float *__restrict__ A, int n, int ld, int m,
                                                          int kchunk, int ntp, float *__restrict__ part) {
  __shared__ Gram6Stage st[2];
  int ti, tj;
  tri_index(blockIdx.x, &ti, &tj);
  const int k0 = blockIdx.y * kchunk;
  const int k1 = min(m, k0 + kchunk);
  float *out = part + ((size_t)blockIdx.y * ntp + blockIdx.x) * kGramTB * kGramTB;
  gram_tile_bf16x6(A, n, ld, ti, tj, k0, k1, st, [&](int r, int c, float v) { out[r * kGramTB + c] = v; });
}

// float64 matrices: the same scheme with 64 x 64 tiles on f64 MFMA.
template <bool TALL>
__global__ __launch_bounds__(256) void gram_f64_kernel(const double *__restrict__ A, int m, int n, int ld,
                                                       int kchunk, int ntp, double *__restrict__ part) {
  constexpr int TB = 64, KC = 16, LS = TB + 2;
  __shared__ double sa[KC][LS];
  __shared__ double sb[KC][LS];
  int ti, tj;
  tri_index(blockIdx.x, &ti, &tj);
  const int kdim = TALL ? m : n;
  const int k0 = blockIdx.y * kchunk;
  const int k1 = min(kdim, k0 + kchunk);
  const int t = threadIdx.x, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  F64Acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64acc_zero();
  for (int kk0 = k0; kk0 < k1; kk0 += KC) {
    for (int f = t; f < KC * TB; f += 256) {
      double va = 0.0, vb = 0.0;
      if (TALL) {
        const int k = f / TB, c = f % TB, row = kk0 + k;
        if (row < k1) {
          if (ti * TB + c < n) va = A[(size_t)row * ld + ti * TB + c];
          if (tj * TB + c < n) vb = A[(size_t)row * ld + tj * TB + c];
        }
        sa[k][c] = va;
        sb[k][c] = vb;
      } else {
        const int r = f % TB, k = f / TB, kc = kk0 + k;
        if (kc < k1) {
          if (ti * TB + r < m) va = A[(size_t)(ti * TB + r) * ld + kc];
          if (tj * TB + r < m) vb = A[(size_t)(tj * TB + r) * ld + kc];
        }
        sa[k][r] = va;
        sb[k][r] = vb;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) f64_tile_step(acc, sa, sb, k4, wi * 32, wj * 32);
    __syncthreads();
  }
  double *out = part + ((size_t)blockIdx.y * ntp + blockIdx.x) * TB * TB;
  f64_tile_store(acc, wi * 32, wj * 32, [&](int r, int c, double v) { out[r * TB + c] = v; });
}

// K = I + sum_splits partials, full symmetric Q x Q (identity in the padding).
// One workgroup per 64 x 64 sub-block of a lower tile: its sums are staged
// in LDS and written twice, as they are (lower half) and transposed (upper
// half), so every write runs along a row of K and both halves hold the same
// bits (those of the lower element).  Sub-blocks wholly above the diagonal
// of a diagonal tile are written by their mirror.
template <typename P>
__global__ __launch_bounds__(256) void gram_reduce_kernel(const P *part, int splits, int ntp, int TB, int q, int Q,
                                                          double *K) {
  __shared__ double tile[64][65];
  const int per = TB / 64, subs = per * per;
  const int tp = blockIdx.x / subs, sub = blockIdx.x % subs;
  int ti, tj;
  tri_index(tp, &ti, &tj);
  const int si = sub / per, sj = sub % per;
  const int i0 = ti * TB + si * 64, j0 = tj * TB + sj * 64;
  if ((ti == tj && si < sj) || i0 >= Q) return;  // uniform over the workgroup
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const P *src = part + (size_t)tp * TB * TB + (size_t)si * 64 * TB + sj * 64;
  const size_t sstride = (size_t)ntp * TB * TB;
  // the thread's 16 rows are summed together, four splits at a time (64
  // loads in flight), each element in split order
  double v[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int i = i0 + ty + 4 * u, j = j0 + tx;
    v[u] = (i == j) ? 1.0 : 0.0;
  }
  const bool jok = j0 + tx < q;
  int s = 0;
  for (; s + 4 <= splits; s += 4) {
    P x[4][16];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const P *ps = src + (s + g) * sstride + tx;
#pragma unroll
      for (int u = 0; u < 16; ++u) x[g][u] = ps[(size_t)(ty + 4 * u) * TB];
    }
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (i0 + ty + 4 * u < q && jok) v[u] += (double)x[g][u];
  }
  for (; s < splits; ++s) {
    const P *ps = src + s * sstride + tx;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = ty + 4 * u;
      if (i0 + r < q && jok) v[u] += (double)ps[(size_t)r * TB];
    }
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) tile[ty + 4 * u][tx] = v[u];
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int i = i0 + r, j = j0 + tx;
    if (i < Q && j < Q && i >= j) K[(size_t)i * Q + j] = tile[r][tx];
    const int it = i0 + tx, jt = j0 + r;  // element (it, jt) of the lower half, stored at (jt, it)
    if (it < Q && jt < Q && it > jt) K[(size_t)jt * Q + it] = tile[tx][r];
  }
}

static void gram_geometry(int m, int n, int elem_size, int *TB, int *ntp, int *splits, int *kchunk) {
  const bool tall = m >= n;
  const int kdim = tall ? m : n, qdim = tall ? n : m;
  *TB = elem_size == 4 ? 128 : 64;
  const int nt = (int)cdiv(qdim, *TB);
  *ntp = nt * (nt + 1) / 2;
  // as many (tile, split) workgroups as are resident at once, one round
  // (two for the tall float32 Gram, below), each split at least 256 deep
  const void *kern = elem_size == 4 ? (tall ? (const void *)gram_bf16x6_kernel : (const void *)gram_f32_kernel<false>)
                                    : (tall ? (const void *)gram_f64_kernel<true> : (const void *)gram_f64_kernel<false>);
  static std::atomic<int> resident[2][2];  // per (element size, orientation); 0 = not yet queried
  int res = resident[elem_size == 4][tall].load(std::memory_order_relaxed);
  if (!res) {
    res = resident_workgroups(kern, elem_size == 4 && tall ? 512 : 256);
    resident[elem_size == 4][tall].store(res, std::memory_order_relaxed);
  }
  int s = (int)std::max<int64_t>(1, std::min<int64_t>(res / *ntp, cdiv(kdim, 256)));
  // the tall float32 Gram takes two rounds of resident workgroups: with one,
  // the tile count leaves up to a fifth of them idle (136 tiles at
  // 20000 x 2000: 3 splits fill 408 of 512), with two the dispatcher refills
  // them, and the shorter splits also accumulate more accurately
  if (elem_size == 4 && tall) s = (int)std::max<int64_t>(1, std::min<int64_t>(2 * (int64_t)res / *ntp, cdiv(kdim, 256)));
  *kchunk = (int)round_up(cdiv(kdim, s), kGramKC);
  *splits = (int)cdiv(kdim, *kchunk);
}

size_t gram_workspace_bytes(int m, int n, int elem_size) {
  int TB, ntp, splits, kchunk;
  gram_geometry(m, n, elem_size, &TB, &ntp, &splits, &kchunk);
  return (size_t)splits * ntp * TB * TB * elem_size;
}

template <typename T>
int run_gram(const T *A, int m, int n, int ld, double *K, int Q, float *ws32, double *ws64, size_t ws_bytes,
             hipStream_t s) {
  int TB, ntp, splits, kchunk;
  gram_geometry(m, n, sizeof(T), &TB, &ntp, &splits, &kchunk);
  if ((size_t)splits * ntp * TB * TB * sizeof(T) > ws_bytes) return POGS_ENOMEM;
  const bool tall = m >= n;
  const int q = std::min(m, n);
  dim3 grid(ntp, splits);
  if constexpr (sizeof(T) == 4) {
    if (tall)
      hipLaunchKernelGGL(gram_bf16x6_kernel, grid, dim3(512), 0, s, (const float *)A, n, ld, m, kchunk, ntp, ws32);
    else
      hipLaunchKernelGGL(gram_f32_kernel<false>, grid, dim3(256), 0, s, (const float *)A, m, n, ld, kchunk, ntp, ws32);
    hipLaunchKernelGGL(gram_reduce_kernel<float>, dim3(ntp * (TB / 64) * (TB / 64)), dim3(256), 0, s, ws32, splits, ntp, TB, q,
                       Q, K);
  } else {
    if (tall)
      hipLaunchKernelGGL(gram_f64_kernel<true>, grid, dim3(256), 0, s, (const double *)A, m, n, ld, kchunk, ntp, ws64);
    else
      hipLaunchKernelGGL(gram_f64_kernel<false>, grid, dim3(256), 0, s, (const double *)A, m, n, ld, kchunk, ntp, ws64);
    hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3(ntp * (TB / 64) * (TB / 64)), dim3(256), 0, s, ws64, splits, ntp, TB, q,
                       Q, K);
  }
  return POGS_OK;
}

// ---------------------------------------------------------------------------
// Blocked Cholesky and explicit inverse (float64, 64 x 64 blocks)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void chol_first_kernel(const double *K, double *B, int Q, double *Dinv,
                                                         unsigned *bad, unsigned *step) {
  __shared__ CholLds cl;
  chol_first_body(K, B, Q, Dinv, bad, step, cl);
}

// L_I0 = K_I0 X_00^T for I > 0 (the panel of step 0).
__global__ __launch_bounds__(256) void chol_panel0_kernel(double *K, int Q, const double *Dinv) {
  __shared__ F64Stage st;
  trsm_tile(K, Q, 0, 1 + blockIdx.x, Dinv, st);
}

template <typename T>
__global__ __launch_bounds__(256, 2) void chol_step_kernel(double *K, double *B, int Q, int nbt, int kb, double *Dinv,
                                                           int q, T *Kinv, int ldk, unsigned *bad, unsigned *step) {
  chol_step_body<T>(blockIdx.x, K, B, Q, nbt, kb, Dinv, q, Kinv, ldk, bad, step);
}

__global__ __launch_bounds__(256) void trtri_init_kernel(double *X, int Q) {
  trtri_init_rows(X, Q, blockIdx.x * 8, min(Q, (int)blockIdx.x * 8 + 8));
}

size_t factor_workspace_bytes(int Q) { return ((size_t)Q * Q + (size_t)Q * NB) * sizeof(double); }

// K (Q x Q, full symmetric I + G; overwritten) -> K^{-1} as T (q x q, row
// stride ldk).  Workspace: B (Q x Q) and the diagonal block inverses (Q x 64).
// bad[0] counts failures; bad[1] is the step flag.
template <typename T>
int run_factor_inverse(double *K, int q, int Q, T *Kinv, int ldk, double *ws, unsigned *bad, hipStream_t s) {
  const int nbt = Q / NB;
  double *B = ws;
  double *Dinv = B + (size_t)Q * Q;
  unsigned *step = bad + 1;
  hipLaunchKernelGGL(trtri_init_kernel, dim3(cdiv(Q, 8)), dim3(256), 0, s, B, Q);
  hipLaunchKernelGGL(chol_first_kernel, dim3(1), dim3(256), 0, s, (const double *)K, B, Q, Dinv, bad, step);
  if (nbt > 1) hipLaunchKernelGGL(chol_panel0_kernel, dim3(nbt - 1), dim3(256), 0, s, K, Q, (const double *)Dinv);
  // padding columns of K^{-1} are read (times zero) by the row-dot kernels: keep them zero
  (void)hipMemsetAsync(Kinv, 0, (size_t)q * ldk * sizeof(T), s);
  const int nupd = nbt * (nbt + 1) / 2;
  for (int kb = 0; kb < nbt; ++kb)
    hipLaunchKernelGGL((chol_step_kernel<T>), dim3(nupd), dim3(256), 0, s, K, B, Q, nbt, kb, Dinv, q, Kinv, ldk, bad,
                       step);
  return POGS_OK;
}

#define POGS_INST(T)                                                                                   \
  template void launch_layout<T>(const void *, pogs_dtype, pogs_order, int64_t, int, int, T *, int,    \
                                 unsigned *, hipStream_t);                                             \
  template int run_equilibrate<T>(T *, int, int, int, int, double, double *, double *, double *,       \
                                  size_t, unsigned *, hipStream_t);                                    \
  template int run_gram<T>(const T *, int, int, int, double *, int, float *, double *, size_t,         \
                           hipStream_t);                                                               \
  template int run_factor_inverse<T>(double *, int, int, T *, int, double *, unsigned *, hipStream_t);
POGS_INST(float)
POGS_INST(double)
#undef POGS_INST

}  // namespace pogs
