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
// float32 A = D A E in 16-byte pieces: thread (x, t) takes columns 4 (256 x
// + t) .. + 3 and rows y, y + ny, ..., four rows in flight.  The same
// arithmetic per entry as scale_matrix_body (D_r A_rc, then times E_c, in
// float64); padding columns (n .. ld) stay zero.
__device__ __forceinline__ void scale_rows_f32_body(const Blk &b, float *A, int m, int n, int ld, const double *D,
                                                    const double *E) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int c4 = (b.x * 256 + (int)threadIdx.x) * 4;
  if (c4 >= n) return;  // c4 + 3 < ld: ld is a multiple of 64
  double e[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) e[k] = c4 + k < n ? E[c4 + k] : 0.0;
  for (int r0 = b.y; r0 < m; r0 += 4 * b.ny) {
    f4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + u * b.ny;
      if (r < m) v[u] = *reinterpret_cast<const f4 *>(A + (size_t)r * ld + c4);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + u * b.ny;
      if (r < m) {
        const double d = D[r];
        f4 o;
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = (float)(d * (double)v[u][k] * e[k]);
        *reinterpret_cast<f4 *>(A + (size_t)r * ld + c4) = o;
      }
    }
  }
}

// Row-major float32 source copied into the row-major layout in 16-byte
// pieces (src 16-byte aligned, lda % 4 == 0): thread (x, t) takes columns
// 4 (256 x + t) .. + 3 of rows y, y + ny, ...; columns n .. ld are zero;
// non-finite entries are counted in *bad.
__device__ __forceinline__ void layout_rows_f32_body(const Blk &b, const float *src, int64_t lda, int m, int n,
                                                     float *dst, int ld, unsigned *bad) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int c4 = (b.x * 256 + (int)threadIdx.x) * 4;
  if (c4 >= ld) return;
  unsigned nbad = 0;
  for (int r0 = b.y; r0 < m; r0 += 4 * b.ny) {
    f4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + u * b.ny;
      v[u] = f4{0.f, 0.f, 0.f, 0.f};
      if (r < m) {
        const float *sp = src + (size_t)r * lda + c4;
        if (c4 + 3 < n) {
          v[u] = *reinterpret_cast<const f4 *>(sp);
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (c4 + k < n) v[u][k] = sp[k];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + u * b.ny;
      if (r < m) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (!isfinite(v[u][k])) ++nbad;
        *reinterpret_cast<f4 *>(dst + (size_t)r * ld + c4) = v[u];
      }
    }
  }
  if (nbad) atomicAdd(bad, nbad);
}

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

// ---------------------------------------------------------------------------
// Blocked Cholesky K = L L^T with L^{-1} and K^{-1} folded in (Section 3.5),
// as the single-problem setup runs it: one launch per step k, in which
//   workgroup 0          factors the next diagonal block I = k + 1 from
//                        K_II - L_Ik L_Ik^T (formed into LDS), stores its
//                        inverse X_II in Dinv block I and in B tile (I, I), and
//                        releases step flag I;
//   trailing workgroups  K_IJ -= L_Ik L_Jk^T (k < J <= I, except (I, I) above);
//                        those of column k + 1 then wait for flag k + 1 and
//                        form L_I,k+1 = K_I,k+1 X_{k+1,k+1}^T in place;
//   inverse workgroups   B_rj -= L_rk X_kj (r > k, j <= k; L X = I by block
//                        forward substitution, B starts as I); those of row
//                        k + 1 then wait for the flag and form
//                        X_k+1,j = X_{k+1,k+1} B_k+1,j in place;
//   K^{-1} workgroups    K^{-1}_IJ += X_kI^T X_kJ (J <= I <= k), adding row k
//                        of X = L^{-1} once it is final (K^{-1} = X^T X).
// So the critical chain of a step is one product, the diagonal factor and
// one product, with no launch between the factor and its panel.
// K^{-1}_IJ (I >= J) accumulates in K's tile (J, I), which the factorisation
// no longer reads (an upper tile, or a diagonal tile already factored); the
// last step writes it as T, mirrored.  Every launch has nbt (nbt + 1) / 2
// workgroups.  Workgroup 0 is dispatched before every workgroup that waits for
// it; a wait gives up after kStepSpin polls and counts a failure in *bad
// (the setup then reports an error) rather than hang.
// ---------------------------------------------------------------------------
constexpr unsigned kStepSpin = 1u << 22;

// Every wave's global stores complete (workgroup scope: they are in the
// device cache), then thread 0 publishes step value v with a device-scope
// release, which writes that cache back once for the whole workgroup.
__device__ inline void step_release(unsigned *step, unsigned v) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(step, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The workgroup's own stores complete first (it reads them back), then thread
// 0 polls for step value >= v with relaxed loads (an acquire per poll would
// invalidate the caches every other workgroup is using) and acquires once at
// device scope when it sees it; the barrier orders the other waves after it.
__device__ inline void step_wait(unsigned *step, unsigned v, unsigned *bad) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned n = 0;
    while (__hip_atomic_load(step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
      __builtin_amdgcn_s_sleep(2);
      if (++n == kStepSpin) {
        atomicAdd(bad, 1u);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// X_II = L_II^{-1} from potrf_diag_core (upper blocks zeroed) into Dinv block
// I and B tile (I, I).
__device__ inline void store_block_inverse(const CholLds &cl, double *Dinv, double *B, int Q, int I) {
  double *dv = Dinv + (size_t)I * NB * NB;
  double *bt = B + (size_t)I * NB * Q + (size_t)I * NB;
#pragma unroll 4
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int r = e / NB, c = e % NB;
    const double v = (c >> 4) > (r >> 4) ? 0.0 : cl.X[r][c];
    dv[e] = v;
    bt[(size_t)r * Q + c] = v;
  }
}

// First diagonal block (before step 0): factor K_00, store X_00, reset the step flag.
__device__ __forceinline__ void chol_first_body(const double *K, double *B, int Q, double *Dinv, unsigned *bad,
                                                unsigned *step, CholLds &cl) {
  constexpr int kPer = NB * NB / 256;
  double v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = threadIdx.x + 256 * u;
    v[u] = K[(size_t)(e / NB) * Q + e % NB];
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = threadIdx.x + 256 * u;
    cl.L[e / NB][e % NB] = v[u];
  }
  __syncthreads();
  potrf_diag_core(cl, bad);
  store_block_inverse(cl, Dinv, B, Q, 0);
  if (threadIdx.x == 0) *step = 0;
}

// Workgroup 0 of step kb: D = K_II - L_I,kb L_I,kb^T (I = kb + 1) into LDS
// (K_II is loaded before the product, in the accumulator's element order),
// its factor and inverse, then step flag I.
__device__ __forceinline__ void chol_next_diag(const double *K, double *B, int Q, int kb, double *Dinv,
                                               unsigned *bad, unsigned *step, F64Stage &st, CholLds &cl) {
  const int I = kb + 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ib = (w >> 1) * 32, jb = (w & 1) * 32;
  const double *C = K + (size_t)I * NB * Q + (size_t)I * NB;
  double c[16];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        c[(i * 2 + j) * 4 + r] = C[(size_t)(ib + i * 16 + 4 * r + (lane >> 4)) * Q + jb + j * 16 + (lane & 15)];
  F64Acc acc[2][2];
  acc_zero(acc);
  const double *LI = K + (size_t)I * NB * Q + (size_t)kb * NB;
  block_product(acc, LI, Q, 1, LI, 1, Q, NB, st);
  int e = 0;
  acc_store(acc, [&](int r, int cc, double v) { cl.L[r][cc] = c[e++] - v; });
  __syncthreads();
  potrf_diag_core(cl, bad);
  store_block_inverse(cl, Dinv, B, Q, I);
  step_release(step, (unsigned)I);
}

template <typename T>
__device__ __forceinline__ void chol_step_body(int b, double *K, double *B, int Q, int nbt, int kb, double *Dinv,
                                               int q, T *Kinv, int ldk, unsigned *bad, unsigned *step) {
  __shared__ union {
    F64Stage st;
    CholLds cl;
  } lds;
  const int rest = nbt - kb - 1;
  const int n0 = rest > 0 ? 1 : 0;              // the next diagonal block
  const int nsy = rest * (rest + 1) / 2 - n0;  // the other trailing tiles
  const int ntr = rest * (kb + 1);              // inverse updates
  if (b < n0) {
    chol_next_diag(K, B, Q, kb, Dinv, bad, step, lds.st, lds.cl);
    return;
  }
  b -= n0;
  if (b < nsy) {
    int I, J;
    tri_index(b + 1, &I, &J);  // trailing tile (0, 0) is workgroup 0's
    I += kb + 1;
    J += kb + 1;
    syrk_tile(K, Q, kb, I, J, lds.st);
    if (J == kb + 1) {
      step_wait(step, (unsigned)J, bad);
      trsm_tile(K, Q, J, I, Dinv, lds.st);
    }
    return;
  }
  b -= nsy;
  if (b < ntr) {
    const int r = kb + 1 + b / (kb + 1), j = b % (kb + 1);
    trtri_update_tile(K, B, Q, kb, r, j, lds.st);
    if (r == kb + 1) {
      step_wait(step, (unsigned)r, bad);
      trtri_scale_tile(Dinv, B, Q, r, j, lds.st);
    }
    return;
  }
  b -= ntr;
  int I, J;
  tri_index(b, &I, &J);  // K^{-1} tile (I, J), J <= I <= kb: += X_kb,I^T X_kb,J
  F64Acc acc[2][2];
  acc_zero(acc);
  const double *Xk = B + (size_t)kb * NB * Q;
  block_product(acc, Xk + (size_t)I * NB, 1, Q, Xk + (size_t)J * NB, Q, 1, NB, lds.st);
  double *S = K + (size_t)J * NB * Q + (size_t)I * NB;
  const bool first = kb == I, last = kb == nbt - 1;
  acc_store(acc, [&](int r, int c, double v) {
    double *p = S + (size_t)r * Q + c;
    const double val = first ? v : *p + v;
    if (!last) {
      *p = val;
      return;
    }
    // a diagonal tile is written from its lower triangle only, so each output
    // element has one writer
    const int gi = I * NB + r, gj = J * NB + c;
    if (gi < q && gj < q && (I != J || r >= c)) {
      Kinv[(size_t)gi * ldk + gj] = (T)val;
      Kinv[(size_t)gj * ldk + gi] = (T)val;
    }
  });
}

template <typename T>
__device__ __forceinline__ void kinv_body(int b, const double *X, int Q, int nbt, int q, T *Kinv, int ldk) {
  __shared__ F64Stage st;
  int I, J;
  tri_index(b, &I, &J);
  kinv_tile<T>(X, Q, nbt, q, Kinv, ldk, I, J, st);
}

}  // namespace pogs
