// Sparse A: the pre-conditioning and the iteration with the CGLS projection
// (Section 3.5) on a matrix kept twice in compressed rows, as A^ and as A^T,
// so both products of a CG step are row passes with no cross-workgroup
// reduction: A^ p is a pass over the rows of A^, A^T [r1, q] one over the
// rows of A^T, and each finishes in its own epilogue.  A CG step is two
// launches (the dense path needs three).
//
// Row pass: a group of lpr lanes per row (lpr chosen from the mean row length)
// walks the row's entries with stride lpr, accumulates in float64 and
// reduces across the group; rows are spread over a grid of at most 1024
// workgroups, whose per-workgroup sums (fixed order) feed the control sums.
#include "cgls.hpp"

namespace pogs {

void sparse_shape(int rows, int64_t nnz, int *lpr, int *grid) {
  const double mean = rows > 0 ? (double)nnz / rows : 0.0;
  int l = 4;
  while (l < 64 && l < mean) l *= 2;
  *lpr = l;
  const int64_t groups = kBlock / l;
  *grid = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(std::max(rows, 1), groups), 1024));
}

int sparse_segment(int m, int n, int64_t nnz, int elem) {
  int64_t nseg = cdiv((int64_t)m, (int64_t)(kSegBytes / (2 * (size_t)elem)));
  nseg = std::max<int64_t>(1, std::min<int64_t>(nseg, nnz / (2 * (int64_t)n)));
  return (int)cdiv((int64_t)m, nseg);
}

void sparse_seg_shape(int rows, int nseg, int64_t nnz, int *lpr, int *grid) {
  int g;
  sparse_shape((int)std::min<int64_t>((int64_t)rows * nseg, 1 << 30), nnz, lpr, &g);
  const int64_t groups = kBlock / *lpr;
  const int64_t want = std::min<int64_t>(cdiv((int64_t)rows, groups), kSegGrid);
  *grid = (int)std::max<int64_t>(1, std::max<int64_t>(want, cdiv((int64_t)rows, (int64_t)kSegRows)));
}

__device__ inline void acc_add(double &a, double b) { a += b; }
__device__ inline void acc_add(Sum2 &a, const Sum2 &b) {
  a.a += b.a;
  a.b += b.b;
}

// Epilogue interface: R row(int i, double s0, double s1) with R double or
// Sum2, and block_done(int block, R sum) in thread 0.  PAIRED: the two
// right-hand sides are interleaved in v0 (v0[2j], v0[2j + 1]).
template <int LPR, int NRHS, bool SQUARE, typename T, typename TV, class Epi, bool PAIRED = false>
__device__ __forceinline__ void spmv_body(const Csr<T> &A, const TV *__restrict__ v0, const TV *__restrict__ v1,
                                          const Epi &epi) {
  typedef TV TV2 __attribute__((ext_vector_type(2)));
  constexpr int G = kBlock / LPR;
  __shared__ double bs[kBlock / kWave];
  const int grp = threadIdx.x / LPR, sub = threadIdx.x % LPR;
  using R = decltype(epi.row(0, 0.0, 0.0));
  R contrib{};
  for (int row = blockIdx.x * G + grp; row < A.rows; row += gridDim.x * G) {
    const int k1 = A.rp[row + 1];
    double s0 = 0.0, s1 = 0.0;
    for (int k = A.rp[row] + sub; k < k1; k += LPR) {
      double a = (double)A.va[k];
      if constexpr (SQUARE) a *= a;
      const int j = A.ci[k];
      if constexpr (PAIRED) {
        const TV2 v = reinterpret_cast<const TV2 *>(v0)[j];
        s0 = fma(a, (double)v.x, s0);
        s1 = fma(a, (double)v.y, s1);
      } else {
        s0 = fma(a, (double)v0[j], s0);
        if constexpr (NRHS > 1) s1 = fma(a, (double)v1[j], s1);
      }
    }
    s0 = group_sum<LPR>(s0);
    if constexpr (NRHS > 1) s1 = group_sum<LPR>(s1);
    if (sub == 0) acc_add(contrib, epi.row(row, s0, s1));
  }
  if constexpr (std::is_same<R, Sum2>::value) {
    const double a = block_sum(contrib.a, bs);
    const double b = block_sum(contrib.b, bs);
    if (threadIdx.x == 0) epi.block_done(blockIdx.x, Sum2{a, b});
  } else {
    const double t = block_sum(contrib, bs);
    if (threadIdx.x == 0) epi.block_done(blockIdx.x, t);
  }
}

// The same pass over the rows of a segmented copy (A^T): every workgroup
// walks the segments in order for its own rows and keeps their sums in LDS,
// so at any moment the grid gathers from one segment's piece of the vector,
// which stays in L2, instead of from the whole m-long vector.  The lane that
// owns a row (sub == 0) is the only one to touch its LDS slot, so the slots
// need no barrier.  Requires ceil(rows / (gridDim.x G)) G <= kSegRows (the
// host's grid does this).
template <int LPR, int NRHS, bool SQUARE, typename T, typename TV, class Epi, bool PAIRED = false>
__device__ __forceinline__ void spmv_seg_body(const Csr<T> &A, const TV *__restrict__ v0, const TV *__restrict__ v1,
                                              const Epi &epi) {
  typedef TV TV2 __attribute__((ext_vector_type(2)));
  constexpr int G = kBlock / LPR;
  __shared__ double acc[NRHS][kSegRows];
  __shared__ double bs[kBlock / kWave];
  const int grp = threadIdx.x / LPR, sub = threadIdx.x % LPR;
  const int first = blockIdx.x * G + grp, stride = gridDim.x * G;
  if (sub == 0)
    for (int row = first, slot = grp; row < A.rows; row += stride, slot += G)
      for (int r = 0; r < NRHS; ++r) acc[r][slot] = 0.0;
  for (int sg = 0; sg < A.nseg; ++sg) {
    const int *__restrict__ rp = A.rp + (size_t)sg * A.rows;
    for (int row = first, slot = grp; row < A.rows; row += stride, slot += G) {
      const int k1 = rp[row + 1];
      double s0 = 0.0, s1 = 0.0;
      for (int k = rp[row] + sub; k < k1; k += LPR) {
        double a = (double)A.va[k];
        if constexpr (SQUARE) a *= a;
        const int j = A.ci[k];
        if constexpr (PAIRED) {
          const TV2 v = reinterpret_cast<const TV2 *>(v0)[j];
          s0 = fma(a, (double)v.x, s0);
          s1 = fma(a, (double)v.y, s1);
        } else {
          s0 = fma(a, (double)v0[j], s0);
          if constexpr (NRHS > 1) s1 = fma(a, (double)v1[j], s1);
        }
      }
      s0 = group_sum<LPR>(s0);
      if constexpr (NRHS > 1) s1 = group_sum<LPR>(s1);
      if (sub == 0) {
        acc[0][slot] += s0;
        if constexpr (NRHS > 1) acc[1][slot] += s1;
      }
    }
  }
  using R = decltype(epi.row(0, 0.0, 0.0));
  R contrib{};
  if (sub == 0)
    for (int row = first, slot = grp; row < A.rows; row += stride, slot += G)
      acc_add(contrib, epi.row(row, acc[0][slot], NRHS > 1 ? acc[NRHS - 1][slot] : 0.0));
  if constexpr (std::is_same<R, Sum2>::value) {
    const double a = block_sum(contrib.a, bs);
    const double b = block_sum(contrib.b, bs);
    if (threadIdx.x == 0) epi.block_done(blockIdx.x, Sum2{a, b});
  } else {
    const double t = block_sum(contrib, bs);
    if (threadIdx.x == 0) epi.block_done(blockIdx.x, t);
  }
}

// A column epilogue of the dense path used on the rows of A^T.
template <class E> struct ColRows {
  E e;
  __device__ Sum2 row(int j, double s0, double s1) const { return e.column(j, s0, s1); }
  __device__ void block_done(int b, const Sum2 &v) const { e.tile_done(b, v.a, v.b); }
};

// ---------------------------------------------------------------------------
// Pre-conditioning
// ---------------------------------------------------------------------------
struct EpiSpEqRow {  // d_i = n / ((A o A) e + gamma/m)_i
  double *d;
  double n, gm;
  __device__ double row(int i, double r, double) const {
    d[i] = n / (r + gm);
    return 0.0;
  }
  __device__ void block_done(int, double) const {}
};
struct EpiSpFro {  // sum_i d_i ((A o A) e)_i = ||sqrt(d) A sqrt(e)||_F^2
  const double *d;
  double *slots;
  __device__ double row(int i, double r, double) const { return d[i] * r; }
  __device__ void block_done(int b, double v) const { slots[b] = v; }
};

template <int LPR, typename T, class Epi, bool SEG>
__global__ __launch_bounds__(kBlock) void sp_square_kernel(Csr<T> A, const double *v, Epi e) {
  if constexpr (SEG) spmv_seg_body<LPR, 1, true, T, double, Epi>(A, v, v, e);
  else spmv_body<LPR, 1, true, T, double, Epi>(A, v, v, e);
}

// SEG: A is the segmented copy of A^T
template <typename T, class Epi, bool SEG>
static void launch_square(const Csr<T> &A, const double *v, const Epi &e, hipStream_t s) {
  const dim3 g(A.grid), b(kBlock);
  switch (A.lpr) {
    case 4: hipLaunchKernelGGL((sp_square_kernel<4, T, Epi, SEG>), g, b, 0, s, A, v, e); break;
    case 8: hipLaunchKernelGGL((sp_square_kernel<8, T, Epi, SEG>), g, b, 0, s, A, v, e); break;
    case 16: hipLaunchKernelGGL((sp_square_kernel<16, T, Epi, SEG>), g, b, 0, s, A, v, e); break;
    case 32: hipLaunchKernelGGL((sp_square_kernel<32, T, Epi, SEG>), g, b, 0, s, A, v, e); break;
    default: hipLaunchKernelGGL((sp_square_kernel<64, T, Epi, SEG>), g, b, 0, s, A, v, e); break;
  }
}

__global__ void sp_fill_kernel(double *v, int len, double x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) v[i] = x;
}

// D = sqrt(d / s), E = sqrt(e / s), s = sqrt(||sqrt(d) A sqrt(e)||_F^2 / min(m, n)).
__global__ __launch_bounds__(kBlock) void sp_eq_finish_kernel(const double *d, const double *e,
                                                              const double *slots, int nslots, int m, int n,
                                                              double *D, double *E) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double fro2 = 0.0;
  for (int t = 0; t < nslots; ++t) fro2 += slots[t];
  const double sc = sqrt(fro2 / (double)min(m, n));
  if (i < m) D[i] = sqrt(d[i] / sc);
  else if (i < m + n) E[i - m] = sqrt(e[i - m] / sc);
}

// A^_ij = D_i A_ij E_j on the rows of A (transposed = false: row r is i) or
// of A^T (transposed = true: row r is j), the same expression in both; one
// wave per row piece (row r % rows of segment r / rows).
template <typename T>
__global__ __launch_bounds__(kBlock) void sp_scale_kernel(Csr<T> A, const double *D, const double *E, bool transposed) {
  const int64_t b = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
  if (b >= (int64_t)A.rows * A.nseg) return;
  const int r = (int)(b % A.rows);
  const int lane = threadIdx.x & (kWave - 1);
  for (int k = A.rp[b] + lane; k < A.rp[b + 1]; k += kWave) {
    const int c = A.ci[k];
    const double di = transposed ? D[c] : D[r], ej = transposed ? E[r] : E[c];
    A.va[k] = (T)(di * (double)A.va[k] * ej);
  }
}

template <typename T>
void run_equilibrate_sparse(Csr<T> A, Csr<T> At, int m, int n, int iters, double eps_cmp, double *D, double *E,
                            double *ws, hipStream_t s) {
  if (iters <= 0) {  // no pre-conditioning: D = E = 1
    hipLaunchKernelGGL(sp_fill_kernel, dim3(cdiv(m, kBlock)), dim3(kBlock), 0, s, D, m, 1.0);
    hipLaunchKernelGGL(sp_fill_kernel, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, E, n, 1.0);
    return;
  }
  double *d = ws, *e = ws + m, *slots = ws + 2 * ((size_t)m + n);
  const double gamma = (double)(m + n) * sqrt(eps_cmp);
  hipLaunchKernelGGL(sp_fill_kernel, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, e, n, 1.0);
  for (int it = 0; it < iters; ++it) {
    launch_square<T, EpiSpEqRow, false>(A, e, EpiSpEqRow{d, (double)n, gamma / m}, s);
    launch_square<T, EpiSpEqRow, true>(At, d, EpiSpEqRow{e, (double)m, gamma / n}, s);
  }
  launch_square<T, EpiSpFro, false>(A, e, EpiSpFro{d, slots}, s);
  hipLaunchKernelGGL(sp_eq_finish_kernel, dim3(cdiv(m + n, kBlock)), dim3(kBlock), 0, s, d, e, slots, A.grid, m, n,
                     D, E);
  hipLaunchKernelGGL(sp_scale_kernel<T>, dim3(cdiv(m, kBlock / kWave)), dim3(kBlock), 0, s, A, D, E, false);
  hipLaunchKernelGGL(sp_scale_kernel<T>, dim3(cdiv((int64_t)n * At.nseg, (int64_t)(kBlock / kWave))), dim3(kBlock), 0,
                     s, At, D, E, true);
}

// ---------------------------------------------------------------------------
// CGLS iteration
// ---------------------------------------------------------------------------
// C0: t = A^ x_h -> r1 = d - t, primal residual sums (the dense epilogue's
// arithmetic), and the pair (r1, nu_h) for the pass over A^T
template <typename T> struct EpiSpStart : EpiBase<T> {
  __device__ double row(int i, double t, double) const {
    const IterArgs<T> &p = this->p;
    const T r1 = (T)((double)p.dy[i] - t);
    p.yt[i] = r1;
    p.pair[2 * (size_t)i] = r1;
    p.pair[2 * (size_t)i + 1] = p.nu[i];
    const double r = t - (double)p.yh[i];
    return r * r;
  }
  __device__ void block_done(int b, double v) const { this->p.s_pri[b] = v; }
};

// KA: the arithmetic of EpiCgRows, and the pair (r1, q_j)
template <typename T> struct EpiSpRows {
  EpiCgRows<T> c;
  __device__ double row(int i, double as, double) const {
    const IterArgs<T> &p = c.p;
    T r1 = p.yt[i];
    double qn = as;
    if (c.has_prev) {
      const double qo = (double)p.qv[i];
      r1 = (T)((double)r1 - c.alpha_prev * qo);
      p.yt[i] = r1;
      qn = as + c.beta * qo;
    }
    const T qt = (T)qn;
    p.qv[i] = qt;
    p.pair[2 * (size_t)i] = r1;
    p.pair[2 * (size_t)i + 1] = qt;
    return (double)qt * (double)qt;
  }
  __device__ void block_done(int b, double v) const { c.p.s_qq[b] = v; }
};

template <int LPR, typename T>
__global__ __launch_bounds__(kBlock) void sp_start_kernel(IterArgs<T> p) {
  EpiSpStart<T> e{{p}};
  if (e.skip()) return;
  spmv_body<LPR, 1, false, T, T, EpiSpStart<T>>(p.sa, p.x, p.x, e);
}

// C1 with its finish: s_0 = A^T r1 + c - x, dual residual sums, ||s_0||^2
template <int LPR, typename T>
__global__ __launch_bounds__(kBlock) void sp_first_kernel(IterArgs<T> p) {
  if (!cg_first_enter<T>(p)) return;
  ColRows<EpiCgFirst<T>> e{EpiCgFirst<T>{p}};
  spmv_seg_body<LPR, 2, false, T, T, ColRows<EpiCgFirst<T>>, true>(p.sat, p.pair, p.pair, e);
}

// KA: q_j = A^ s_j + beta q_{j-1}, pending r1 update
template <int LPR, typename T>
__global__ __launch_bounds__(kBlock) void sp_rows_kernel(IterArgs<T> p, int j, int cap) {
  EpiSpRows<T> e;
  if (!cg_rows_enter<T>(p, j, cap, &e.c)) return;
  spmv_body<LPR, 1, false, T, T, EpiSpRows<T>>(p.sa, p.sv, p.sv, e);
}

// KB and KC together: A^T [r1, q_j] on the rows of A^T, then p_j, x, s_{j+1}
template <int LPR, typename T>
__global__ __launch_bounds__(kBlock) void sp_step_kernel(IterArgs<T> p, int j) {
  EpiCgStep<T> e;
  if (!cg_step_enter<T>(p, j, &e)) return;
  ColRows<EpiCgStep<T>> c{e};
  spmv_seg_body<LPR, 2, false, T, T, ColRows<EpiCgStep<T>>, true>(p.sat, p.pair, p.pair, c);
}

#define POGS_SP_DISPATCH(lpr, KERNEL, grid, s, ...)                                                        \
  switch (lpr) {                                                                                            \
    case 4: hipLaunchKernelGGL((KERNEL<4, T>), dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__); break;         \
    case 8: hipLaunchKernelGGL((KERNEL<8, T>), dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__); break;         \
    case 16: hipLaunchKernelGGL((KERNEL<16, T>), dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__); break;       \
    case 32: hipLaunchKernelGGL((KERNEL<32, T>), dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__); break;       \
    default: hipLaunchKernelGGL((KERNEL<64, T>), dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__); break;       \
  }

template <typename T> static void launch_sp_first(const IterArgs<T> &p, hipStream_t s) {
  POGS_SP_DISPATCH(p.sa.lpr, sp_start_kernel, p.sa.grid, s, p)
  POGS_SP_DISPATCH(p.sat.lpr, sp_first_kernel, p.sat.grid, s, p)
}

template <typename T> static void launch_sp_rows(const IterArgs<T> &p, int j, int cap, hipStream_t s) {
  POGS_SP_DISPATCH(p.sa.lpr, sp_rows_kernel, p.sa.grid, s, p, j, cap)
}

template <typename T> static void launch_sp_step(const IterArgs<T> &p, int j, int cap, hipStream_t s) {
  launch_sp_rows<T>(p, j, cap, s);
  POGS_SP_DISPATCH(p.sat.lpr, sp_step_kernel, p.sat.grid, s, p, j)
}

template <typename T> void launch_iteration_cg_sparse(const IterArgs<T> &p, int cap, hipStream_t s) {
  launch_prox_cg<T>(p, s);
  launch_sp_first<T>(p, s);
  for (int j = 0; j < cap; ++j) launch_sp_step<T>(p, j, cap, s);
  launch_sp_rows<T>(p, cap, cap, s);
}

template <typename T> void launch_iteration_cg_sparse_part(const IterArgs<T> &p, int which, hipStream_t s) {
  if (which == 0) launch_prox_cg<T>(p, s);
  else if (which == 1) launch_sp_first<T>(p, s);
  else launch_sp_step<T>(p, 0, 1 << 30, s);
}

// Warm start (the dense path's change of variables): x = E^-1 x0, y = A^ x
// over the rows of A^, y~ = -(D^-1 nu0) / rho0, x~ = -A^T y~ over the rows
// of A^T.
template <typename T> struct EpiSpWarm {
  T *out;
  double sign;
  __device__ double row(int i, double v, double) const {
    out[i] = (T)(sign * v);
    return 0.0;
  }
  __device__ void block_done(int, double) const {}
};

template <int LPR, typename T>
__global__ __launch_bounds__(kBlock) void sp_warm_kernel(Csr<T> A, const T *v, EpiSpWarm<T> e) {
  spmv_body<LPR, 1, false, T, T, EpiSpWarm<T>>(A, v, v, e);
}
template <int LPR, typename T>
__global__ __launch_bounds__(kBlock) void sp_warm_seg_kernel(Csr<T> A, const T *v, EpiSpWarm<T> e) {
  spmv_seg_body<LPR, 1, false, T, T, EpiSpWarm<T>>(A, v, v, e);
}

template <typename T>
void launch_warm_start_sparse(const IterArgs<T> &p, const double *D, const double *E, double rho0, const T *x0,
                              const T *nu0, hipStream_t s) {
  if (x0) {
    hipLaunchKernelGGL(warm_scale_kernel<T>, dim3(cdiv(p.n, kBlock)), dim3(kBlock), 0, s, x0, E, true, 1.0, p.n,
                       p.x);
    POGS_SP_DISPATCH(p.sa.lpr, sp_warm_kernel, p.sa.grid, s, p.sa, (const T *)p.x, EpiSpWarm<T>{p.y, 1.0})
  }
  // the missing half estimated as in the dense warm start (one proximal point step)
  if (nu0) {
    hipLaunchKernelGGL(warm_scale_kernel<T>, dim3(cdiv(p.m, kBlock)), dim3(kBlock), 0, s, nu0, D, true,
                       -1.0 / rho0, p.m, p.yt);
  } else if (x0) {
    hipLaunchKernelGGL(warm_estimate_kernel<T>, dim3(cdiv(p.m, kBlock)), dim3(kBlock), 0, s, p.f, (const T *)p.y,
                       p.yt, p.m, (T)rho0, 0);
  }
  if (nu0 || x0)
    POGS_SP_DISPATCH(p.sat.lpr, sp_warm_seg_kernel, p.sat.grid, s, p.sat, (const T *)p.yt, EpiSpWarm<T>{p.xt, -1.0})
  if (nu0 && !x0) {
    hipLaunchKernelGGL(warm_estimate_kernel<T>, dim3(cdiv(p.n, kBlock)), dim3(kBlock), 0, s, p.g, (const T *)p.xt,
                       p.x, p.n, (T)rho0, 1);
    POGS_SP_DISPATCH(p.sa.lpr, sp_warm_kernel, p.sa.grid, s, p.sa, (const T *)p.x, EpiSpWarm<T>{p.y, 1.0})
  }
}

#undef POGS_SP_DISPATCH

#define POGS_INST(T)                                                                                        \
  template void run_equilibrate_sparse<T>(Csr<T>, Csr<T>, int, int, int, double, double *, double *,        \
                                          double *, hipStream_t);                                           \
  template void launch_iteration_cg_sparse<T>(const IterArgs<T> &, int, hipStream_t);                       \
  template void launch_iteration_cg_sparse_part<T>(const IterArgs<T> &, int, hipStream_t);                  \
  template void launch_warm_start_sparse<T>(const IterArgs<T> &, const double *, const double *, double,      \
                                            const T *, const T *, hipStream_t);
POGS_INST(float)
POGS_INST(double)
#undef POGS_INST

}  // namespace pogs
