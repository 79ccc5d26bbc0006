// Workgroup-level building blocks of the setup (256 threads = 4 waves):
//   * Gram tiles on f32 MFMA (128 x 128 output tile, 4 waves in 2 x 2),
//   * float64 64 x 64 block products on f64 MFMA,
//   * the diagonal-block Cholesky / triangular inverse, panel solve, trailing
//     update, blocked inverse steps and the K^{-1} = L^{-T} L^{-1} product.
// The multi-workgroup setup launches one workgroup per tile; the batched
// solver calls the same functions in loops inside one workgroup per problem.
#pragma once

#include "common.hpp"
#include "mfma.hpp"

namespace pogs {

constexpr int NB = 64;        // Cholesky block size
constexpr int LSF = NB + 2;   // row stride of the float64 LDS stages

struct F64Stage {             // 16.9 KB
  double a[16][LSF];
  double b[16][LSF];
};
struct CholLds {              // 68.6 KB
  double L[NB][NB + 1];
  double X[NB][NB + 1];
  double red[4][NB];
};
constexpr int kGramTB = 128;  // f32 Gram tile
struct GramStage {            // 16.9 KB
  float a[16][kGramTB + 4];
  float b[16][kGramTB + 4];
};

// Tile pair t of a lower triangle (ti >= tj), row by row.
__device__ inline void tri_index(int t, int *ti, int *tj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  *ti = i;
  *tj = t - i * (i + 1) / 2;
}

typedef float GramAcc __attribute__((ext_vector_type(4)));

// Gram tile (ti, tj) over k in [k0, k1): TALL: sum_k A[k][i] A[k][j] (A^T A),
// else sum_k A[i][k] A[j][k] (A A^T).  Each wave owns a 64 x 64 quarter as
// 4 x 4 f32 MFMA 16x16x4 blocks; out(row, col, value) visits the tile's
// elements (tile-local indices).  Reads beyond m / n are zero.
template <bool TALL, class Out>
__device__ void gram_tile_f32(const float *__restrict__ A, int m, int n, int ld, int ti, int tj, int k0, int k1,
                              GramStage &st, Out out) {
  constexpr int TB = kGramTB, KC = 16;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  const bool diag = ti == tj;
  typedef float f4 __attribute__((ext_vector_type(4)));
  GramAcc acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = GramAcc{0.f, 0.f, 0.f, 0.f};

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
        *reinterpret_cast<f4 *>(&st.a[k][c]) = va;
        if (!diag) *reinterpret_cast<f4 *>(&st.b[k][c]) = vb;
      } else {
        const int r = f & 127, kq = (f >> 7) * 4;
        const int kc = kk0 + kq;  // kc + 3 < ld (kk0 % 16 == 0, ld % 64 == 0, kk0 < n <= ld)
        const int ra = ti * TB + r, rb = tj * TB + r;
        f4 va = f4{0.f, 0.f, 0.f, 0.f}, vb = f4{0.f, 0.f, 0.f, 0.f};
        if (ra < m) va = *reinterpret_cast<const f4 *>(A + (size_t)ra * ld + kc);
        if (!diag && rb < m) vb = *reinterpret_cast<const f4 *>(A + (size_t)rb * ld + kc);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool ok = kc + u < k1;
          st.a[kq + u][r] = ok ? va[u] : 0.f;
          if (!diag) st.b[kq + u][r] = ok ? vb[u] : 0.f;
        }
      }
    }
    __syncthreads();
    const float(*pb)[TB + 4] = diag ? st.a : st.b;
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      float av[4], bv[4];
      const int kr = k4 + (lane >> 4), cl = lane & 15;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        av[b] = st.a[kr][wi * 64 + b * 16 + cl];
        bv[b] = pb[kr][wj * 64 + b * 16 + cl];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // f32 16x16x4 result layout: lane l, element r -> row 4 (l / 16) + r, column l % 16
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out(wi * 64 + i * 16 + 4 * (lane >> 4) + r, wj * 64 + j * 16 + (lane & 15), acc[i][j][r]);
}

// General f32 MFMA tile product: tile (i0.., j0..) of sum_{k in [k0, k1)} opA(i, k) B(k, j)
// with opA(i, k) = A[k * lda + i] (A_T: A stored K x M) or A[i * lda + k]
// (A stored M x K), B stored K x N row-major (ldb % 4 == 0).  Rows >= M,
// columns >= N and k >= k1 read as zero; lda and ldb are multiples of 4 and
// the rows of A and B are readable up to the next multiple of 16 elements
// past M (A_T), k1 (not A_T) and N.  out(row, col, value) gets tile-local
// indices.  128 x 128 tile, 4 waves in 2 x 2, f32 MFMA 16x16x4.
template <bool A_T, class Out>
__device__ void gemm_tile_f32(const float *__restrict__ A, int lda, int M, const float *__restrict__ B, int ldb,
                              int N, int i0, int j0, int k0, int k1, GramStage &st, Out out) {
  constexpr int TB = kGramTB, KC = 16;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  typedef float f4 __attribute__((ext_vector_type(4)));
  GramAcc acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = GramAcc{0.f, 0.f, 0.f, 0.f};
  for (int kk0 = k0; kk0 < k1; kk0 += KC) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int f = t + h * 256;  // float4 index in a 16 x 128 stage
      // B: rows kk0 + k, columns j0 + c .. c + 3
      {
        const int k = f >> 5, c = (f & 31) * 4;
        const int row = kk0 + k, col = j0 + c;
        f4 vb = f4{0.f, 0.f, 0.f, 0.f};
        if (row < k1 && col < N) vb = *reinterpret_cast<const f4 *>(B + (size_t)row * ldb + col);
        *reinterpret_cast<f4 *>(&st.b[k][c]) = vb;
      }
      if (A_T) {
        const int k = f >> 5, c = (f & 31) * 4;
        const int row = kk0 + k, col = i0 + c;
        f4 va = f4{0.f, 0.f, 0.f, 0.f};
        if (row < k1 && col < M) va = *reinterpret_cast<const f4 *>(A + (size_t)row * lda + col);
        *reinterpret_cast<f4 *>(&st.a[k][c]) = va;
      } else {
        const int r = f & 127, kq = (f >> 7) * 4;
        const int row = i0 + r, kc = kk0 + kq;
        f4 va = f4{0.f, 0.f, 0.f, 0.f};
        if (row < M && kc < k1) va = *reinterpret_cast<const f4 *>(A + (size_t)row * lda + kc);
#pragma unroll
        for (int u = 0; u < 4; ++u) st.a[kq + u][r] = kc + u < k1 ? va[u] : 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      float av[4], bv[4];
      const int kr = k4 + (lane >> 4), cl = lane & 15;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        av[b] = st.a[kr][wi * 64 + b * 16 + cl];
        bv[b] = st.b[kr][wj * 64 + b * 16 + cl];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out(wi * 64 + i * 16 + 4 * (lane >> 4) + r, wj * 64 + j * 16 + (lane & 15), acc[i][j][r]);
}

// acc += sum_{k < K} opA(i, k) opB(k, j) for a 64 x 64 float64 tile, with
// opA(i, k) = pa[i * sai + k * sak], opB(k, j) = pb[k * sbk + j * sbj]
// (K a multiple of 16).  Ends with a barrier: the stages may be reused and
// the operands overwritten afterwards.
__device__ inline void block_product(F64Acc acc[2][2], const double *pa, int64_t sai, int64_t sak, const double *pb,
                                     int64_t sbk, int64_t sbj, int K, F64Stage &st) {
  const int t = threadIdx.x, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int f = t; f < 16 * NB; f += 256) {
      const int k = f / NB, i = f % NB;
      st.a[k][i] = pa[(int64_t)i * sai + (int64_t)(k0 + k) * sak];
      st.b[k][i] = pb[(int64_t)(k0 + k) * sbk + (int64_t)i * sbj];
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) f64_tile_step<LSF>(acc, st.a, st.b, k4, wi * 32, wj * 32);
    __syncthreads();
  }
}

__device__ inline void acc_zero(F64Acc acc[2][2]) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f64acc_zero();
}

template <class Fn> __device__ inline void acc_store(const F64Acc acc[2][2], Fn fn) {
  const int w = threadIdx.x >> 6;
  f64_tile_store(acc, (w >> 1) * 32, (w & 1) * 32, fn);
}

// Factor diagonal block kb of K (Q x Q, row-major, lower) and invert the
// factor, in LDS with the whole workgroup (4 waves).  Left-looking Cholesky:
// at step j, row r needs v_r = K_rj - sum_{k<j} L_rk L_jk; wave w sums the
// terms k in [16w, 16w + 16), wave 0 adds the four partial sums in wave order,
// takes the pivot L_jj = sqrt(v_j) from lane j and stores L_rj = v_r / L_jj.
// The inverse X = L^{-1} is built row by row the same way:
// X_rc = (delta_rc - sum_{c<=q<r} L_rq X_qc) / L_rr for all columns c at once.
// Writes L_kk (upper part zeroed) back into K and L_kk^{-1} into Dinv block
// kb.  A non-positive pivot counts in *bad and is replaced by 1.
__device__ inline void potrf_diag(double *K, int Q, int kb, double *Dinv, unsigned *bad, CholLds &s) {
  const int t = threadIdx.x;
  const int lane = t & 63, part = t >> 6;
  double *blk = K + (size_t)kb * NB * Q + (size_t)kb * NB;
  for (int e = t; e < NB * NB; e += blockDim.x) s.L[e / NB][e % NB] = blk[(size_t)(e / NB) * Q + e % NB];
  __syncthreads();
  const int k0 = part * 16;
  unsigned nbad = 0;
  for (int j = 0; j < NB; ++j) {
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int kk = 0; kk < 16; kk += 2) {
      if (k0 + kk < j) a0 = fma(s.L[lane][k0 + kk], s.L[j][k0 + kk], a0);
      if (k0 + kk + 1 < j) a1 = fma(s.L[lane][k0 + kk + 1], s.L[j][k0 + kk + 1], a1);
    }
    s.red[part][lane] = a0 + a1;
    __syncthreads();
    if (part == 0) {
      const double v = s.L[lane][j] - ((s.red[0][lane] + s.red[1][lane]) + (s.red[2][lane] + s.red[3][lane]));
      double piv = __shfl(v, j, 64);
      if (!(piv > 0.0) || !isfinite(piv)) {
        ++nbad;
        piv = 1.0;
      }
      const double d = sqrt(piv);
      if (lane == j) s.L[lane][j] = d;
      else if (lane > j) s.L[lane][j] = v / d;
    }
    __syncthreads();
  }
  if (nbad && t == 0) atomicAdd(bad, nbad);
  for (int rr = 0; rr < NB; ++rr) {
    // partial sums over q in [16 part, 16 part + 16) with c <= q < rr, column c = lane
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int kk = 0; kk < 16; kk += 2) {
      const int q0 = k0 + kk, q1 = q0 + 1;
      if (q0 < rr && q0 >= lane) a0 = fma(s.L[rr][q0], s.X[q0][lane], a0);
      if (q1 < rr && q1 >= lane) a1 = fma(s.L[rr][q1], s.X[q1][lane], a1);
    }
    s.red[part][lane] = a0 + a1;
    __syncthreads();
    if (part == 0) {
      const double acc = (s.red[0][lane] + s.red[1][lane]) + (s.red[2][lane] + s.red[3][lane]);
      s.X[rr][lane] = lane > rr ? 0.0 : ((rr == lane ? 1.0 : 0.0) - acc) / s.L[rr][rr];
    }
    __syncthreads();
  }
  double *dv = Dinv + (size_t)kb * NB * NB;
  for (int e = t; e < NB * NB; e += blockDim.x) {
    const int r = e / NB, c = e % NB;
    blk[(size_t)r * Q + c] = c <= r ? s.L[r][c] : 0.0;
    dv[e] = s.X[r][c];
  }
  __syncthreads();
}

// L_ib,kb = K_ib,kb L_kb,kb^{-T}   (in place)
__device__ inline void trsm_tile(double *K, int Q, int kb, int ib, const double *Dinv, F64Stage &st) {
  double *blk = K + (size_t)ib * NB * Q + (size_t)kb * NB;
  const double *dv = Dinv + (size_t)kb * NB * NB;
  F64Acc acc[2][2];
  acc_zero(acc);
  block_product(acc, blk, Q, 1, dv, 1, NB, NB, st);
  acc_store(acc, [&](int r, int c, double v) { blk[(size_t)r * Q + c] = v; });
}

// K_I,J -= L_I,kb L_J,kb^T
__device__ inline void syrk_tile(double *K, int Q, int kb, int I, int J, F64Stage &st) {
  const double *LI = K + (size_t)I * NB * Q + (size_t)kb * NB;
  const double *LJ = K + (size_t)J * NB * Q + (size_t)kb * NB;
  double *C = K + (size_t)I * NB * Q + (size_t)J * NB;
  F64Acc acc[2][2];
  acc_zero(acc);
  block_product(acc, LI, Q, 1, LJ, 1, Q, NB, st);
  acc_store(acc, [&](int r, int c, double v) { C[(size_t)r * Q + c] -= v; });
}

// Blocked L^{-1} by right-looking block forward substitution of L X = I:
// X holds B = I - sum_{k<i} L_.k X_k. (initialised to the identity); step i
// sets X_ij = L_ii^{-1} B_ij for j <= i (trtri_scale_tile), then
// B_rj -= L_ri X_ij for r > i, j <= i (trtri_update_tile).  Every launch of a
// step is many independent 64 x 64 x 64 products.
__device__ inline void trtri_scale_tile(const double *Dinv, double *X, int Q, int i, int j, F64Stage &st) {
  F64Acc acc[2][2];
  acc_zero(acc);
  double *C = X + (size_t)i * NB * Q + (size_t)j * NB;
  block_product(acc, Dinv + (size_t)i * NB * NB, NB, 1, C, Q, 1, NB, st);
  acc_store(acc, [&](int r, int c, double v) { C[(size_t)r * Q + c] = v; });
}

__device__ inline void trtri_update_tile(const double *K, double *X, int Q, int i, int r, int j, F64Stage &st) {
  F64Acc acc[2][2];
  acc_zero(acc);
  const double *pa = K + (size_t)r * NB * Q + (size_t)i * NB;  // L_ri
  const double *pb = X + (size_t)i * NB * Q + (size_t)j * NB;  // X_ij
  block_product(acc, pa, Q, 1, pb, Q, 1, NB, st);
  double *C = X + (size_t)r * NB * Q + (size_t)j * NB;
  acc_store(acc, [&](int rr, int cc, double v) { C[(size_t)rr * Q + cc] -= v; });
}

// X <- I on the lower block triangle, diagonal blocks included whole (the
// block products read full 64 x 64 blocks; blocks above the diagonal are
// never read).
__device__ inline void trtri_init_rows(double *X, int Q, int row0, int row1) {
  for (int i = row0; i < row1; ++i) {
    const int jend = (i / NB + 1) * NB;
    for (int j = threadIdx.x; j < jend; j += blockDim.x) X[(size_t)i * Q + j] = i == j ? 1.0 : 0.0;
  }
}

// K^{-1}_I,J = sum_{k >= I} X_k,I^T X_k,J for I >= J, written and mirrored as T
// (entries of index >= q skipped).
template <typename T>
__device__ inline void kinv_tile(const double *X, int Q, int nbt, int q, T *Kinv, int ldk, int I, int J,
                                 F64Stage &st) {
  F64Acc acc[2][2];
  acc_zero(acc);
  const double *pa = X + (size_t)I * NB * Q + (size_t)I * NB;
  const double *pb = X + (size_t)I * NB * Q + (size_t)J * NB;
  block_product(acc, pa, 1, Q, pb, Q, 1, (nbt - I) * NB, st);
  acc_store(acc, [&](int r, int c, double v) {
    const int gi = I * NB + r, gj = J * NB + c;
    if (gi < q && gj < q) {
      Kinv[(size_t)gi * ldk + gj] = (T)v;
      Kinv[(size_t)gj * ldk + gi] = (T)v;
    }
  });
}

}  // namespace pogs
