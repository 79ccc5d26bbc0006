// One-time setup per matrix, on gfx950:
//   layout      : host/device A (f32/f64, row/col-major) -> row-major T, ld % 64 == 0
//   equilibrate : Algorithm 2 (regularised Sinkhorn-Knopp, p = 2,
//                 gamma = (m + n) sqrt(eps_cmp)) for a fixed sweep count, then
//                 the Frobenius normalisation of Section 4.1.2 and A <- D A E
//   gram        : G = A^T A (m >= n) or A A^T (m < n) on MFMA (f32 MFMA with
//                 f32 accumulation inside a K split; splits summed in f64),
//                 K = I + G in float64 (Section 3.5)
//   factor      : blocked Cholesky K = L L^T in float64 (64 x 64 blocks, f64
//                 MFMA for the block products), L^{-1} by blocked substitution,
//                 K^{-1} = L^{-T} L^{-1}, stored in T for the iterations.
#include "gemv.hpp"
#include "internal.hpp"
#include "mfma.hpp"

namespace pogs {

// ---------------------------------------------------------------------------
// Layout conversion
// ---------------------------------------------------------------------------
template <typename T, typename S>
__global__ __launch_bounds__(256) void layout_kernel(const S *src, int colmajor, int64_t lda, int m,
                                                     int n, T *dst, int ld, unsigned *bad) {
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  unsigned nbad = 0;
  if (colmajor) {
    // read down columns (coalesced along rows), write along rows
    for (int k = ty; k < 32; k += 8) {
      const int c = c0 + k, r = r0 + tx;
      T v = T(0);
      if (r < m && c < n) {
        const double x = (double)src[(size_t)c * lda + r];
        if (!isfinite(x)) ++nbad;
        v = (T)x;
      }
      tile[k][tx] = v;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
      const int r = r0 + k, c = c0 + tx;
      if (r < m && c < ld) dst[(size_t)r * ld + c] = tile[tx][k];
    }
  } else {
    for (int k = ty; k < 32; k += 8) {
      const int r = r0 + k, c = c0 + tx;
      if (r < m && c < ld) {
        T v = T(0);
        if (c < n) {
          const double x = (double)src[(size_t)r * lda + c];
          if (!isfinite(x)) ++nbad;
          v = (T)x;
        }
        dst[(size_t)r * ld + c] = v;
      }
    }
  }
  if (nbad) atomicAdd(bad, nbad);
}

template <typename T>
void launch_layout(const void *src, pogs_dtype sdt, pogs_order ord, int64_t lda, int m, int n, T *dst,
                   int ld, unsigned *bad, hipStream_t s) {
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
struct EqArgs {
  double *d, *e, *colsum, *slots, *fro2;
  double gamma_m, gamma_n;  // gamma / m, gamma / n
  double mf, nf;            // m, n as doubles
};

// d_i = n / (sum_j A_ij^2 e_j + gamma/m)
struct EpiEqRow {
  EqArgs a;
  static constexpr bool kFinal = false;
  __device__ bool skip() const { return false; }
  __device__ double row(int i, double s, double) const { a.d[i] = a.nf / (s + a.gamma_m); return 0.0; }
  __device__ void block_done(int, double) const {}
  __device__ void final(double *) const {}
};

// e_j = m / (sum_i A_ij^2 d_i + gamma/n); also sum_j e_j colsum_j = ||D A E||_F^2
struct EpiEqCol {
  EqArgs a;
  static constexpr bool kFinal = true;
  __device__ bool skip() const { return false; }
  __device__ double column(int j, double s, double) const {
    const double e = a.mf / (s + a.gamma_n);
    a.e[j] = e;
    return e * s;
  }
  __device__ void tile_done(int tile, double v) const { a.slots[tile] = v; }
  __device__ void final(double *lds) const {
    double t = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) t += load_agent(a.slots + i);
    const double tot = block_sum(t, lds);
    if (threadIdx.x == 0) *a.fro2 = tot;
  }
};

__global__ void fill_kernel(double *p, double v, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = v;
}

// D_i = sqrt(d_i / s), E_j = sqrt(e_j / s) with s = sqrt(fro2 / q): the
// Frobenius norm of D A E over sqrt(min(m, n)) becomes 1 (Section 4.1.2).
__global__ void equil_finish_kernel(const double *d, const double *e, const double *fro2, int m, int n,
                                    int q, double *D, double *E) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double s = sqrt(*fro2 / (double)q);
  if (i < m) D[i] = sqrt(d[i] / s);
  else if (i < m + n) E[i - m] = sqrt(e[i - m] / s);
}

// A <- D A E in place (padding columns stay zero).
template <typename T>
__global__ void scale_matrix_kernel(T *A, int m, int n, int ld, const double *D, const double *E) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  for (int r = blockIdx.y; r < m; r += gridDim.y) A[(size_t)r * ld + c] = (T)(D[r] * (double)A[(size_t)r * ld + c] * E[c]);
}

size_t equil_workspace_bytes(int m, int n) {
  int splits, rps, ncolp;
  gemv_t_geometry(m, n, 4, &splits, &rps, &ncolp);
  int s2, r2, nc2;
  gemv_t_geometry(m, n, 8, &s2, &r2, &nc2);
  const size_t part = (size_t)std::max(splits * ncolp, s2 * nc2);
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
  unsigned *tile_cnt = counters;  // counters holds tiles + 1 (zeroed) entries
  unsigned *fin_cnt = counters + tiles;
  for (int it = 0; it < iters; ++it) {
    // rows: d = n / (|A|^2 e + gamma/m)
    {
      EpiEqRow er{a};
      constexpr int VN = Vec16<T>::N;
      if (cdiv(n, VN) >= 128)
        hipLaunchKernelGGL((gemv_n_kernel<T, double, 1, true, 64, 1, EpiEqRow>),
                           dim3(cdiv(m, gemv_n_rows_per_block<64, 1>())), dim3(kBlock), 0, s, A, m, n, ld,
                           a.e, a.e, fin_cnt, er);
      else
        hipLaunchKernelGGL((gemv_n_kernel<T, double, 1, true, 16, 1, EpiEqRow>),
                           dim3(cdiv(m, gemv_n_rows_per_block<16, 1>())), dim3(kBlock), 0, s, A, m, n, ld,
                           a.e, a.e, fin_cnt, er);
    }
    // columns: e = m / (|A^T|^2 d + gamma/n)
    {
      EpiEqCol ec{a};
      hipLaunchKernelGGL((gemv_t_kernel<T, double, 1, true, EpiEqCol>), dim3(tiles, splits), dim3(kBlock),
                         0, s, A, m, n, ld, a.d, a.d, rps, part, ncolp, tile_cnt, fin_cnt, ec);
    }
  }
  const int q = std::min(m, n);
  hipLaunchKernelGGL(equil_finish_kernel, dim3(cdiv(m + n, 256)), dim3(256), 0, s, a.d, a.e, a.fro2, m, n, q,
                     D, E);
  hipLaunchKernelGGL((scale_matrix_kernel<T>), dim3(cdiv(n, 256), std::min(m, 32768)), dim3(256), 0, s, A, m, n,
                     ld, D, E);
  return POGS_OK;
}

// ---------------------------------------------------------------------------
// Gram matrix on MFMA
// ---------------------------------------------------------------------------
// Tile pair t of the lower triangle (ti >= tj).
__device__ inline void tri_index(int t, int *ti, int *tj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  *ti = i;
  *tj = t - i * (i + 1) / 2;
}

// G tile (ti, tj) partial over the K range of split blockIdx.y.
// TALL: G = A^T A, k runs over rows; else G = A A^T, k runs over columns.
// float: 128 x 128 tile, 4 waves in 2 x 2, each 64 x 64 = 4 x 4 MFMA 16x16x4 f32.
template <bool TALL>
__global__ __launch_bounds__(256) void gram_f32_kernel(const float *__restrict__ A, int m, int n, int ld,
                                                       int kchunk, int ntp, float *__restrict__ part) {
  constexpr int TB = 128, KC = 16, LS = TB + 4;
  __shared__ float sa[KC][LS];
  __shared__ float sb[KC][LS];
  int ti, tj;
  tri_index(blockIdx.x, &ti, &tj);
  const int kdim = TALL ? m : n;
  const int qdim = TALL ? n : m;
  const int k0 = blockIdx.y * kchunk;
  const int k1 = min(kdim, k0 + kchunk);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  const bool diag = ti == tj;
  typedef float f4 __attribute__((ext_vector_type(4)));
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  for (int kk0 = k0; kk0 < k1; kk0 += KC) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int f = t + h * 256;  // float4 index in the 16 x 128 stage
      if (TALL) {
        const int k = f >> 5, c = (f & 31) * 4;
        const int row = kk0 + k;
        f4 va = f4{0.f, 0.f, 0.f, 0.f}, vb = f4{0.f, 0.f, 0.f, 0.f};
        if (row < k1) {
          const int ca = ti * TB + c, cb = tj * TB + c;
          if (ca < n) va = *reinterpret_cast<const f4 *>(A + (size_t)row * ld + ca);
          if (!diag && cb < n) vb = *reinterpret_cast<const f4 *>(A + (size_t)row * ld + cb);
        }
        *reinterpret_cast<f4 *>(&sa[k][c]) = va;
        if (!diag) *reinterpret_cast<f4 *>(&sb[k][c]) = vb;
      } else {
        const int r = f & 127, kq = (f >> 7) * 4;
        const int kc = kk0 + kq;  // kc + 3 < ld always (kk0 % 16 == 0, ld % 64 == 0, kk0 < n <= ld)
        const int ra = ti * TB + r, rb = tj * TB + r;
        f4 va = f4{0.f, 0.f, 0.f, 0.f}, vb = f4{0.f, 0.f, 0.f, 0.f};
        if (ra < m) va = *reinterpret_cast<const f4 *>(A + (size_t)ra * ld + kc);
        if (!diag && rb < m) vb = *reinterpret_cast<const f4 *>(A + (size_t)rb * ld + kc);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool ok = kc + u < k1;
          sa[kq + u][r] = ok ? va[u] : 0.f;
          if (!diag) sb[kq + u][r] = ok ? vb[u] : 0.f;
        }
      }
    }
    __syncthreads();
    const float(*pb)[LS] = diag ? sa : sb;
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      float av[4], bv[4];
      const int kr = k4 + (lane >> 4), cl = lane & 15;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        av[b] = sa[kr][wi * 64 + b * 16 + cl];
        bv[b] = pb[kr][wj * 64 + b * 16 + cl];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  float *out = part + ((size_t)blockIdx.y * ntp + blockIdx.x) * TB * TB;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wi * 64 + i * 16 + 4 * (lane >> 4) + r;
        const int col = wj * 64 + j * 16 + (lane & 15);
        out[row * TB + col] = acc[i][j][r];
      }
  (void)qdim;
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
template <typename P>
__global__ void gram_reduce_kernel(const P *part, int splits, int ntp, int TB, int q, int Q, double *K) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= Q) return;
  double v = (i == j) ? 1.0 : 0.0;
  if (i < q && j < q) {
    const int a = max(i, j), b = min(i, j);
    const int ti = a / TB, tj = b / TB;
    const int tp = ti * (ti + 1) / 2 + tj;
    const int ri = a % TB, cj = b % TB;
    for (int s = 0; s < splits; ++s) v += (double)part[((size_t)s * ntp + tp) * TB * TB + ri * TB + cj];
  }
  K[(size_t)i * Q + j] = v;
}

static void gram_geometry(int m, int n, int elem_size, int *TB, int *ntp, int *splits, int *kchunk) {
  const bool tall = m >= n;
  const int kdim = tall ? m : n, qdim = tall ? n : m;
  *TB = elem_size == 4 ? 128 : 64;
  const int nt = (int)cdiv(qdim, *TB);
  *ntp = nt * (nt + 1) / 2;
  int s = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(512, *ntp), cdiv(kdim, 256)));
  *kchunk = (int)round_up(cdiv(kdim, s), 16);
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
      hipLaunchKernelGGL(gram_f32_kernel<true>, grid, dim3(256), 0, s, (const float *)A, m, n, ld, kchunk, ntp, ws32);
    else
      hipLaunchKernelGGL(gram_f32_kernel<false>, grid, dim3(256), 0, s, (const float *)A, m, n, ld, kchunk, ntp, ws32);
    hipLaunchKernelGGL(gram_reduce_kernel<float>, dim3(cdiv(Q, 256), Q), dim3(256), 0, s, ws32, splits, ntp, TB, q,
                       Q, K);
  } else {
    if (tall)
      hipLaunchKernelGGL(gram_f64_kernel<true>, grid, dim3(256), 0, s, (const double *)A, m, n, ld, kchunk, ntp, ws64);
    else
      hipLaunchKernelGGL(gram_f64_kernel<false>, grid, dim3(256), 0, s, (const double *)A, m, n, ld, kchunk, ntp, ws64);
    hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3(cdiv(Q, 256), Q), dim3(256), 0, s, ws64, splits, ntp, TB, q,
                       Q, K);
  }
  return POGS_OK;
}

// ---------------------------------------------------------------------------
// Blocked Cholesky and explicit inverse (float64, 64 x 64 blocks)
// ---------------------------------------------------------------------------
constexpr int NB = 64;

// Factor the diagonal block kb in LDS (unblocked right-looking Cholesky) and
// invert the triangular factor by column substitution.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double *K, int Q, int kb, double *Dinv, unsigned *bad) {
  __shared__ double L[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int t = threadIdx.x;
  double *blk = K + (size_t)kb * NB * Q + (size_t)kb * NB;
  for (int e = t; e < NB * NB; e += 256) L[e / NB][e % NB] = blk[(size_t)(e / NB) * Q + e % NB];
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    if (t == 0) {
      double v = L[j][j];
      if (!(v > 0.0) || !isfinite(v)) {
        atomicAdd(bad, 1u);
        v = 1.0;
      }
      L[j][j] = sqrt(v);
    }
    __syncthreads();
    const double djj = L[j][j];
    for (int r = j + 1 + t; r < NB; r += 256) L[r][j] /= djj;
    __syncthreads();
    const int nr = NB - 1 - j;
    for (int e = t; e < nr * nr; e += 256) {
      const int r = j + 1 + e / nr, c = j + 1 + e % nr;
      if (c <= r) L[r][c] -= L[r][j] * L[c][j];
    }
    __syncthreads();
  }
  if (t < NB) {
    const int c = t;
    for (int r = 0; r < c; ++r) X[r][c] = 0.0;
    X[c][c] = 1.0 / L[c][c];
    for (int r = c + 1; r < NB; ++r) {
      double s = 0.0;
      for (int k = c; k < r; ++k) s += L[r][k] * X[k][c];
      X[r][c] = -s / L[r][r];
    }
  }
  __syncthreads();
  double *dv = Dinv + (size_t)kb * NB * NB;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    blk[(size_t)r * Q + c] = c <= r ? L[r][c] : 0.0;
    dv[e] = X[r][c];
  }
}

// Generic 64 x 64 float64 block product on MFMA:
//   C = beta C + alpha sum_k opA(i, k) opB(k, j), k in [0, K)
// with opA(i, k) = pa[i * sai + k * sak] and opB(k, j) = pb[k * sbk + j * sbj].
__device__ void block_product(F64Acc acc[2][2], const double *pa, int64_t sai, int64_t sak, const double *pb,
                              int64_t sbk, int64_t sbj, int K, double (*sa)[NB + 2], double (*sb)[NB + 2]) {
  const int t = threadIdx.x, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int f = t; f < 16 * NB; f += 256) {
      const int k = f / NB, i = f % NB;
      sa[k][i] = pa[(int64_t)i * sai + (int64_t)(k0 + k) * sak];
      sb[k][i] = pb[(int64_t)(k0 + k) * sbk + (int64_t)i * sbj];
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) f64_tile_step(acc, sa, sb, k4, wi * 32, wj * 32);
    __syncthreads();
  }
}

// L_ik = K_ik L_kk^{-T} for block rows i > kb.
__global__ __launch_bounds__(256) void trsm_panel_kernel(double *K, int Q, int kb, const double *Dinv) {
  __shared__ double sa[16][NB + 2];
  __shared__ double sb[16][NB + 2];
  const int ib = kb + 1 + blockIdx.x;
  double *blk = K + (size_t)ib * NB * Q + (size_t)kb * NB;
  const double *dv = Dinv + (size_t)kb * NB * NB;
  F64Acc acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f64acc_zero();
  // out(r, c) = sum_t K_ik(r, t) Dinv(c, t)
  block_product(acc, blk, Q, 1, dv, 1, NB, NB, sa, sb);
  const int w = threadIdx.x >> 6;
  f64_tile_store(acc, (w >> 1) * 32, (w & 1) * 32, [&](int r, int c, double v) { blk[(size_t)r * Q + c] = v; });
}

// K_IJ -= L_Ik L_Jk^T for kb < J <= I.
__global__ __launch_bounds__(256) void syrk_update_kernel(double *K, int Q, int kb) {
  __shared__ double sa[16][NB + 2];
  __shared__ double sb[16][NB + 2];
  int I, J;
  tri_index(blockIdx.x, &I, &J);
  I += kb + 1;
  J += kb + 1;
  const double *LI = K + (size_t)I * NB * Q + (size_t)kb * NB;
  const double *LJ = K + (size_t)J * NB * Q + (size_t)kb * NB;
  double *C = K + (size_t)I * NB * Q + (size_t)J * NB;
  F64Acc acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f64acc_zero();
  block_product(acc, LI, Q, 1, LJ, 1, Q, NB, sa, sb);
  __syncthreads();
  const int w = threadIdx.x >> 6;
  f64_tile_store(acc, (w >> 1) * 32, (w & 1) * 32,
                 [&](int r, int c, double v) { C[(size_t)r * Q + c] -= v; });
}

// X_ii = L_ii^{-1}
__global__ void inv_diag_copy_kernel(const double *Dinv, double *X, int Q, int nbt) {
  const int b = blockIdx.x;
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x)
    X[(size_t)(b * NB + e / NB) * Q + b * NB + e % NB] = Dinv[(size_t)b * NB * NB + e];
  (void)nbt;
}

// Step i of L^{-1} by blocks: X_ij <- sum_{k=j}^{i-1} L_ik X_kj  (j < i)
__global__ __launch_bounds__(256) void inv_accum_kernel(const double *K, double *X, int Q, int ib) {
  __shared__ double sa[16][NB + 2];
  __shared__ double sb[16][NB + 2];
  const int jb = blockIdx.x;
  F64Acc acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f64acc_zero();
  const double *pa = K + (size_t)ib * NB * Q + (size_t)jb * NB;  // L_i,j.. (row ib, cols from jb)
  const double *pb = X + (size_t)jb * NB * Q + (size_t)jb * NB;  // X_j..,j
  block_product(acc, pa, Q, 1, pb, Q, 1, (ib - jb) * NB, sa, sb);
  double *C = X + (size_t)ib * NB * Q + (size_t)jb * NB;
  const int w = threadIdx.x >> 6;
  f64_tile_store(acc, (w >> 1) * 32, (w & 1) * 32, [&](int r, int c, double v) { C[(size_t)r * Q + c] = v; });
}

// X_ij <- -L_ii^{-1} X_ij (in place, j < i)
__global__ __launch_bounds__(256) void inv_scale_kernel(const double *Dinv, double *X, int Q, int ib) {
  __shared__ double sa[16][NB + 2];
  __shared__ double sb[16][NB + 2];
  const int jb = blockIdx.x;
  F64Acc acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f64acc_zero();
  double *C = X + (size_t)ib * NB * Q + (size_t)jb * NB;
  block_product(acc, Dinv + (size_t)ib * NB * NB, NB, 1, C, Q, 1, NB, sa, sb);
  __syncthreads();
  const int w = threadIdx.x >> 6;
  f64_tile_store(acc, (w >> 1) * 32, (w & 1) * 32, [&](int r, int c, double v) { C[(size_t)r * Q + c] = -v; });
}

// K^{-1}_IJ = sum_{k >= I} X_kI^T X_kJ for I >= J; written (and mirrored) as T.
template <typename T>
__global__ __launch_bounds__(256) void kinv_kernel(const double *X, int Q, int nbt, int q, T *Kinv, int ldk) {
  __shared__ double sa[16][NB + 2];
  __shared__ double sb[16][NB + 2];
  int I, J;
  tri_index(blockIdx.x, &I, &J);
  F64Acc acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f64acc_zero();
  const double *pa = X + (size_t)I * NB * Q + (size_t)I * NB;  // (i, k) -> X[(I*NB + k) * Q + I*NB + i]
  const double *pb = X + (size_t)I * NB * Q + (size_t)J * NB;  // (k, j) -> X[(I*NB + k) * Q + J*NB + j]
  block_product(acc, pa, 1, Q, pb, Q, 1, (nbt - I) * NB, sa, sb);
  const int w = threadIdx.x >> 6;
  f64_tile_store(acc, (w >> 1) * 32, (w & 1) * 32, [&](int r, int c, double v) {
    const int gi = I * NB + r, gj = J * NB + c;
    if (gi < q && gj < q) {
      Kinv[(size_t)gi * ldk + gj] = (T)v;
      Kinv[(size_t)gj * ldk + gi] = (T)v;
    }
  });
}

template <typename T>
int run_factor_inverse(double *K, int q, int Q, T *Kinv, int ldk, double *ws, unsigned *bad, hipStream_t s) {
  const int nbt = Q / NB;
  double *X = ws;                        // Q x Q
  double *Dinv = ws + (size_t)Q * Q;     // nbt blocks of 64 x 64
  for (int kb = 0; kb < nbt; ++kb) {
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, K, Q, kb, Dinv, bad);
    const int rest = nbt - kb - 1;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_panel_kernel, dim3(rest), dim3(256), 0, s, K, Q, kb, (const double *)Dinv);
      hipLaunchKernelGGL(syrk_update_kernel, dim3(rest * (rest + 1) / 2), dim3(256), 0, s, K, Q, kb);
    }
  }
  hipLaunchKernelGGL(inv_diag_copy_kernel, dim3(nbt), dim3(256), 0, s, (const double *)Dinv, X, Q, nbt);
  for (int ib = 1; ib < nbt; ++ib) {
    hipLaunchKernelGGL(inv_accum_kernel, dim3(ib), dim3(256), 0, s, (const double *)K, X, Q, ib);
    hipLaunchKernelGGL(inv_scale_kernel, dim3(ib), dim3(256), 0, s, (const double *)Dinv, X, Q, ib);
  }
  // padding columns of K^{-1} are read (times zero) by the row-dot kernels: keep them zero
  (void)hipMemsetAsync(Kinv, 0, (size_t)q * ldk * sizeof(T), s);
  hipLaunchKernelGGL((kinv_kernel<T>), dim3(nbt * (nbt + 1) / 2), dim3(256), 0, s, (const double *)X, Q, nbt, q,
                     Kinv, ldk);
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
