// Device-side pieces of the one-time setup shared by the single-problem
// launches (setup.hip) and the grouped launches over many problems
// (group.hip): layout conversion, the Sinkhorn-Knopp sweep and Frobenius
// normalisation (Algorithm 2, Section 4.1.2), the blocked Cholesky and
// inverse steps and K^{-1} (Section 3.5).  Every body takes its block
// coordinates explicitly.
#pragma once

#include "factor.hpp"
#include "gemv.hpp"
#include "internal.hpp"

namespace pogs {

template <typename T, typename S>
__device__ __forceinline__ void layout_body(const Blk &b, const S *src, int colmajor, int64_t lda, int m, int n,
                                            T *dst, int ld, unsigned *bad) {
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int r0 = b.y * 32, c0 = b.x * 32;
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

struct EqArgs {
  double *d, *e, *colsum, *slots, *fro2;
  double gamma_m, gamma_n;  // gamma / m, gamma / n
  double mf, nf;            // m, n as doubles
};

// d_i = n / (sum_j A_ij^2 e_j + gamma/m)
struct EpiEqRow {
  EqArgs a;
  __device__ bool skip() const { return false; }
  __device__ double row(int i, double s, double) const { a.d[i] = a.nf / (s + a.gamma_m); return 0.0; }
  __device__ void block_done(int, double) const {}
};

// e_j = m / (sum_i A_ij^2 d_i + gamma/n); the per-tile sums of e_j colsum_j
// give ||D A E||_F^2 after the last sweep.
struct EpiEqCol {
  EqArgs a;
  __device__ bool skip() const { return false; }
  __device__ double column(int j, double s, double) const {
    const double e = a.mf / (s + a.gamma_n);
    a.e[j] = e;
    return e * s;
  }
  __device__ void tile_done(int tile, double v) const { a.slots[tile] = v; }
};

// One Sinkhorn-Knopp sweep (Algorithm 2, p = 2) in a single pass over a
// float32 A with n <= 1024 U: workgroup b owns rows [b rps, (b + 1) rps) and
// thread t the columns 4 t + 1024 u.  For each group of R rows the row sums
// sum_j A_ij^2 e_j are reduced across the workgroup (fixed order: lane tree,
// then waves in order), every thread forms d_i = n / (sum + gamma/m) and adds
// A_ij^2 d_i to its column sums while the row is still in registers.  The
// column sums of each workgroup go to part[b * ncolp + j]; a finish kernel
// adds them in workgroup order and forms e.  Same arithmetic as the two-pass
// sweep, half the reads of A.
template <int U, int R>
__device__ __forceinline__ void equil_sweep_body(const Blk &b, const float *__restrict__ A, int m, int n, int ld,
                                                 int rps, const double *__restrict__ e, double *__restrict__ d,
                                                 double *__restrict__ part, int ncolp, double nf, double gamma_m) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  __shared__ double red[2][R][kBlock / kWave];
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t >> 6;
  const int r0 = b.x * rps, r1 = min(m, r0 + rps);
  double ev[U][4], col[U][4];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = 4 * t + 1024 * u + k;
      ev[u][k] = c < n ? e[c] : 0.0;
      col[u][k] = 0.0;
    }
  int g = 0;
  for (int i0 = r0; i0 < r1; i0 += R, ++g) {
    f4 a[R][U];
#pragma unroll
    for (int ri = 0; ri < R; ++ri) {
      const int row = min(i0 + ri, r1 - 1);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = 4 * t + 1024 * u;
        a[ri][u] = c < ld ? *reinterpret_cast<const f4 *>(A + (size_t)row * ld + c) : f4{0.f, 0.f, 0.f, 0.f};
      }
    }
    double p[R];
#pragma unroll
    for (int ri = 0; ri < R; ++ri) {
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double x = (double)a[ri][u][k];
          acc = fma(x * x, ev[u][k], acc);
        }
      p[ri] = wave_sum(acc);
    }
    if (lane == 0)
#pragma unroll
      for (int ri = 0; ri < R; ++ri) red[g & 1][ri][w] = p[ri];
    __syncthreads();
#pragma unroll
    for (int ri = 0; ri < R; ++ri) {
      const double rs = ((red[g & 1][ri][0] + red[g & 1][ri][1]) + red[g & 1][ri][2]) + red[g & 1][ri][3];
      const bool live = i0 + ri < r1;
      const double di = live ? nf / (rs + gamma_m) : 0.0;
      if (t == 0 && live) d[i0 + ri] = di;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double x = (double)a[ri][u][k];
          col[u][k] = fma(x * x, di, col[u][k]);
        }
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = 4 * t + 1024 * u + k;
      if (c < ncolp) part[(size_t)b.x * ncolp + c] = col[u][k];
    }
}

// D_i = sqrt(d_i / s), E_j = sqrt(e_j / s) with s = sqrt(fro2 / q): the
// Frobenius norm of D A E over sqrt(min(m, n)) becomes 1 (Section 4.1.2).
__device__ __forceinline__ void equil_finish_body(const Blk &b, const double *d, const double *e,
                                                  const double *slots, int ntiles, int m, int n, int q, double *D,
                                                  double *E) {
  const int i = b.x * 256 + threadIdx.x;
  double fro2 = 0.0;
  for (int t = 0; t < ntiles; ++t) fro2 += slots[t];
  const double s = sqrt(fro2 / (double)q);
  if (i < m) D[i] = sqrt(d[i] / s);
  else if (i < m + n) E[i - m] = sqrt(e[i - m] / s);
}

// A <- D A E in place (padding columns stay zero).
template <typename T>
__device__ __forceinline__ void scale_matrix_body(const Blk &b, T *A, int m, int n, int ld, const double *D,
                                                  const double *E) {
  const int c = b.x * 256 + threadIdx.x;
  if (c >= n) return;
  for (int r = b.y; r < m; r += b.ny) A[(size_t)r * ld + c] = (T)(D[r] * (double)A[(size_t)r * ld + c] * E[c]);
}

// Step kb, first half: panel solve L_ib,kb = K_ib,kb L_kb,kb^{-T} for ib > kb
// (workgroups [0, rest)) and the blocked-inverse step X_kb,j = L_kb,kb^{-1} B_kb,j
// for j <= kb (workgroups [rest, rest + kb + 1)).  The two groups touch
// disjoint blocks.
__device__ __forceinline__ void factor_panel_body(int b, double *K, double *X, int Q, int nbt, int kb,
                                                  const double *Dinv) {
  __shared__ F64Stage st;
  const int rest = nbt - kb - 1;
  if (b < rest) trsm_tile(K, Q, kb, kb + 1 + b, Dinv, st);
  else trtri_scale_tile(Dinv, X, Q, kb, b - rest, st);
}

// Step kb, second half: trailing update K_I,J -= L_I,kb L_J,kb^T for
// kb < J <= I (workgroups [0, T)), the workgroup of the next diagonal block
// then factors it (saving a launch per step); and the blocked-inverse update
// B_r,j -= L_r,kb X_kb,j for r > kb, j <= kb (workgroups [T, T + rest (kb + 1))),
// which reads block column kb of L, untouched by the trailing update.
__device__ __forceinline__ void factor_update_body(int b, double *K, double *X, int Q, int nbt, int kb, double *Dinv,
                                                   unsigned *bad) {
  __shared__ union {
    F64Stage st;
    CholLds cl;
  } lds;
  const int rest = nbt - kb - 1;
  const int T = rest * (rest + 1) / 2;
  if (b < T) {
    int I, J;
    tri_index(b, &I, &J);
    syrk_tile(K, Q, kb, I + kb + 1, J + kb + 1, lds.st);
    if (b == 0) {
      __syncthreads();
      potrf_diag(K, Q, kb + 1, Dinv, bad, lds.cl);
    }
  } else {
    const int w = b - T;
    trtri_update_tile(K, X, Q, kb, kb + 1 + w / (kb + 1), w % (kb + 1), lds.st);
  }
}

template <typename T>
__device__ __forceinline__ void kinv_body(int b, const double *X, int Q, int nbt, int q, T *Kinv, int ldk) {
  __shared__ F64Stage st;
  int I, J;
  tri_index(b, &I, &J);
  kinv_tile<T>(X, Q, nbt, q, Kinv, ldk, I, J, st);
}

}  // namespace pogs
